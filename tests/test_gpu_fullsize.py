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


def test_fullsize_bf16x_iteration_matches_oracle(lib, pair):
    """One whole iteration at 50k from the late state with K = 300 imported
    eigenpairs (a seeded orthonormal basis and a decaying spectrum, so the
    oracle needs no 50k eigensolve): E-step, Fast M-step (eq. 20), sigma^2
    (eq. 18 with P').  Transformed points to 1e-3 relative RMS, sigma^2 to
    1e-3 relative."""
    import torch
    X, Y = _f32(pair.X), _f32(pair.Y)
    M = X.shape[0]
    K = 300
    rng = np.random.default_rng(11)
    U, _ = np.linalg.qr(rng.normal(size=(M, K)))
    lam = np.sort(M * 0.5 ** (np.arange(K) / 12.0))[::-1].copy()
    Xt, s2 = _f32(pair.Y_hat), 7.1e-4
    say("fullsize iteration K", K, "sigma2", s2)
    r = lib.Registration(dev(X, torch.float32), dev(Y, torch.float32), precision="bf16x",
                         beta=pair.beta, lam=pair.lam, w=pair.w, eig_mode="import", K=K,
                         tol=0.0, max_iter=10)
    r.prepare(U=dev(U, torch.float64), lam=dev(lam, torch.float64))
    r.set_state(dev(Xt, torch.float32), s2)
    r.step()
    Xg, _, s2g = r.state()
    es = cpd64.estep(Xt, Y, s2, pair.w)
    _, Xo = cpd64.fast_mstep(X, es.Yt, U, lam, pair.lam, s2)
    s2o = cpd64.sigma2_fast(Xt, Y, s2, es, Xo)
    err = cpd64.rel_rms(host(Xg), Xo)
    say("Xt rel_rms", err, "sigma2", s2g, s2o, "rel", abs(s2g - s2o) / s2o)
    assert err < 1e-3
    assert abs(s2g - s2o) < 1e-3 * s2o


def test_fullsize_topk_eigenpairs(lib, pair):
    """The randomized top-K eigensolver at 50k in the benchmark's setting
    (K = 300, oversampling 20, two power steps): orthonormal vectors,
    eigenvalues in descending order within [0, trace Phi = M], and on 64
    sampled rows of Phi (formed directly) residuals |Phi u - lam u| below
    1e-9 lam_1 for every eigenpair above 1e-8 lam_1."""
    import torch
    X, Y = _f32(pair.X), _f32(pair.Y)
    M = X.shape[0]
    r = lib.Registration(dev(X, torch.float32), dev(Y, torch.float32), precision="bf16x",
                         beta=pair.beta, lam=pair.lam, w=pair.w, eig_mode="topk", K=300,
                         oversample=20, power_iters=2, seed=0)
    r.prepare()
    U, lam = (host(t) for t in r.export_eig())
    say("fullsize topk lam_1", lam[0], "lam_K", lam[-1])
    assert np.all(np.diff(lam) <= 0) and lam[-1] >= -1e-9 * lam[0] and lam.sum() <= M
    G = U.T @ U
    assert np.abs(G - np.eye(U.shape[1])).max() < 1e-10
    rows = np.sort(np.random.default_rng(3).choice(M, 64, replace=False))
    Phr = np.exp(-cpd64.sqdist(X[rows], X) / (2.0 * pair.beta ** 2))
    big = lam > 1e-8 * lam[0]
    res = Phr @ U[:, big] - U[rows][:, big] * lam[big]
    say("eigenpairs above 1e-8 lam_1:", int(big.sum()), "max residual / lam_1",
        float(np.abs(res).max() / lam[0]))
    assert np.abs(res).max() < 1e-9 * lam[0]
