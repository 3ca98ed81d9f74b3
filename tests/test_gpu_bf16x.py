"""BF16X precision mode (E-step squared distances from bf16 matrix-core
products with fp32 accumulation) against the FP64 oracle.  Bar: 1e-3
relative RMS on transformed points, as for every reduced-precision mode."""
import numpy as np
import pytest

import synth
from oracle import cpd64, eig64
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

TOL = 1e-3


def _f32(a):
    return a.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("M,N,w,s2", [(700, 1333, 0.1, 0.01), (257, 3001, 0.2, 0.5),
                                      (1025, 513, 0.0, 0.02), (1, 1, 0.1, 0.1),
                                      (4000, 3900, 0.2, 0.001)])
def test_bf16x_estep(lib, M, N, w, s2):
    import torch
    say("bf16x estep", M, N, w, s2)
    rng = np.random.default_rng(M + N)
    Y = _f32(rng.normal(0, 1, (N, 3)))
    X = _f32(Y[rng.choice(N, M, replace=M > N)] + rng.normal(0, 0.05, (M, 3)))
    r = lib.Registration(dev(X, torch.float32), dev(Y, torch.float32), precision="bf16x",
                         beta=1.0, lam=2.0, w=w, eig_mode="import", K=1)
    r.set_state(dev(X, torch.float32), s2)
    g = r.estep()
    es = cpd64.estep(X, Y, s2, w)
    err = cpd64.rel_rms(host(g["Yt"]), es.Yt)
    say("Yt rel_rms", err)
    assert err < TOL
    np.testing.assert_allclose(host(g["logd"]), es.logd, rtol=0, atol=1e-2 * max(1, np.abs(es.logd).max()))
    np.testing.assert_allclose(host(g["P1"]), es.P1, rtol=1e-2, atol=1e-30)
    # sum p |y - x|^2 / P1 from the row-sum product's columns (sum p |y|^2,
    # sum p y, sum p); each term carries the exponent error of the split-bf16
    # distance (up to ~1% here: kappa |x|^2 reaches ~1e4 at sigma^2 = 1e-3)
    np.testing.assert_allclose(host(g["tbar"]), es.tbar, rtol=2e-2, atol=1e-3 * es.tbar.mean())


def test_bf16x_far_rows_and_empty_columns_take_the_exact_path(lib):
    """A model point 300 units from the scene (its row underflows) and, with
    w = 0, a scene point at 160 sigma from every model point (its column
    underflows): both take the exact path inside the merges, and the column's
    refreshed L_n must reach pass B's scene features."""
    import torch
    X = np.array([[0.0, 0, 0], [0.05, 0, 0], [300.0, 0, 0], [0, 0.02, 0]])
    Y = np.array([[0.01, 0, 0], [-0.02, 0, 0], [0, 0.03, 0], [0, -5.0, 0], [2.0, 0, 0]])
    for w in (0.0, 0.1):
        say("bf16x far rows", w)
        r = lib.Registration(dev(X, torch.float32), dev(Y, torch.float32), precision="bf16x",
                             beta=1.0, lam=2.0, w=w, eig_mode="import", K=1)
        r.set_state(dev(X, torch.float32), 1e-3)
        g = r.estep()
        es = cpd64.estep(X, Y, 1e-3, w)
        Yt = host(g["Yt"])
        assert np.all(np.isfinite(Yt))
        err = cpd64.rel_rms(Yt, es.Yt)
        say("Yt rel_rms", err)
        # as in FP32: without the sink the lone column's exponents are ~1.8e4
        assert err < (TOL if w > 0 else 2e-3)
        np.testing.assert_allclose(host(g["logd"]), es.logd, rtol=0,
                                   atol=1e-2 * max(1, np.abs(es.logd).max()))
        np.testing.assert_allclose(host(g["P1"]), es.P1, rtol=1e-2, atol=1e-30)


def test_bf16x_matches_fp32_closely(lib):
    """The split-bf16 cross term carries 24 significant bits: at moderate
    sigma^2 the BF16X E-step agrees with the fp32 direct-difference one far
    inside the 1e-3 bar."""
    import torch
    say("bf16x vs fp32")
    p = synth.surface_pair(M=5000, N=5200, seed=8)
    X, Y = _f32(p.X), _f32(p.Y)
    out, tb = {}, {}
    for prec in ("fp32", "bf16x"):
        r = lib.Registration(dev(X, torch.float32), dev(Y, torch.float32), precision=prec,
                             beta=p.beta, lam=p.lam, w=p.w, eig_mode="import", K=1)
        r.set_state(dev(X, torch.float32), 0.005)
        g = r.estep()
        out[prec] = host(g["Yt"])
        tb[prec] = host(g["tbar"])
    err = cpd64.rel_rms(out["bf16x"], out["fp32"])
    err_t = float(np.abs(tb["bf16x"] - tb["fp32"]).max() / tb["fp32"].mean())
    say("bf16x vs fp32", err, "tbar", err_t)
    assert err < 1e-4
    assert err_t < 5e-3


def test_bf16x_registration(lib):
    """20 EM iterations on a noisy 3000-point surface pair (GPU top-K eig),
    against the oracle with the same test matrix."""
    import torch
    say("bf16x registration")
    p = synth.surface_pair(M=3000, N=3100, seed=5, beta=1.5, lam=2.0, w=0.7,
                           outlier_frac=0.2, noise=0.02)
    X, Y = _f32(p.X), _f32(p.Y)
    K, over = 200, 20
    Om = synth.gaussian_matrix(p.M, K + over, seed=4)
    Uo, lo = eig64.eig_topk(X, p.beta, K, Om, power_iters=2)
    ref = cpd64.register(X, Y, p.beta, p.lam, p.w, "fast", eig=(Uo, lo), iters=20)
    r = lib.Registration(dev(X, torch.float32), dev(Y, torch.float32), precision="bf16x",
                         beta=p.beta, lam=p.lam, w=p.w, eig_mode="topk", K=K, oversample=over,
                         tol=0.0, max_iter=20)
    out = r.prepare(omega=dev(Om, torch.float64)).register()
    err = cpd64.rel_rms(host(out.Xt), ref.Xt)
    say("rel_rms", err, "sigma2", out.sigma2, ref.sigma2)
    assert out.iters == 20 and err < TOL
