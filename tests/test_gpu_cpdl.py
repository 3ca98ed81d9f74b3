"""CPD-L (eq. 21 with the rank-K Gram of eq. 19) on the GPU against the
oracle's cpdl_mstep: one step from the same state with the same (imported)
eigenpairs, FP64 1e-10 and FP32 1e-5 relative RMS on Xt; 30 FP64 iterations;
and the randomized top-K eigen-prep end to end."""
import numpy as np
import pytest

import synth
from oracle import cpd64, eig64
from tests.gpu_util import dev, host, say, torch_dtype

pytestmark = pytest.mark.gpu


def _f32(a):
    return a.astype(np.float32).astype(np.float64)


def _topk(X, beta, K):
    lam, U = np.linalg.eigh(eig64.gram(X, beta))
    o = np.argsort(lam)[::-1][:K]
    return np.ascontiguousarray(U[:, o]), lam[o]


@pytest.mark.parametrize("precision,M,N,K", [("fp64", 700, 650, 60), ("fp32", 1000, 1100, 100),
                                             ("fp64", 300, 5, 300), ("fp32", 129, 257, 7)])
def test_one_cpdl_step(lib, precision, M, N, K):
    import torch
    say("cpdl one step", precision, M, N, K)
    p = synth.sphere_pair(M=M, N=N, seed=M + K)
    X, Y = (p.X, p.Y) if precision == "fp64" else (_f32(p.X), _f32(p.Y))
    U, lam = _topk(X, p.beta, K)
    rng = np.random.default_rng(4)
    Xt = X + 0.03 * rng.normal(size=X.shape)
    if precision == "fp32":
        Xt = _f32(Xt)
    s2 = 0.05
    dt = torch_dtype(precision)
    r = lib.Registration(dev(X, dt), dev(Y, dt), precision=precision, method="cpdl",
                         eig_mode="import", K=K, beta=p.beta, lam=p.lam, w=p.w)
    r.prepare(dev(U, torch.float64), dev(lam, torch.float64))
    r.set_state(dev(Xt, dt), s2)
    r.step()
    Xg, Wg, s2g = r.state()
    es = cpd64.estep(Xt, Y, s2, p.w)
    W, Xn = cpd64.cpdl_mstep(X, es.P1, es.PY, U, lam, p.lam, s2)
    s2n = cpd64.sigma2_cpd(Xt, Y, s2, es, Xn)
    tol = 1e-10 if precision == "fp64" else 1e-5
    err = cpd64.rel_rms(host(Xg), Xn)
    say("rel_rms", err, "sigma2", s2g, s2n)
    assert err < tol
    assert s2g == pytest.approx(s2n, rel=10 * tol)


def test_cpdl_thirty_iterations_fp64(lib):
    import torch
    say("cpdl small500 x30")
    p = synth.workload("small500")
    U, lam = _topk(p.X, p.beta, 50)
    ref = cpd64.register(p.X, p.Y, p.beta, p.lam, p.w, "cpdl", eig=(U, lam), iters=30)
    r = lib.Registration(dev(p.X, torch.float64), dev(p.Y, torch.float64), precision="fp64",
                         method="cpdl", eig_mode="import", K=50, beta=p.beta, lam=p.lam, w=p.w,
                         tol=0.0, max_iter=30)
    out = r.prepare(dev(U, torch.float64), dev(lam, torch.float64)).register()
    err = cpd64.rel_rms(host(out.Xt), ref.Xt)
    say("rel_rms", err, "sigma2", out.sigma2, ref.sigma2)
    assert out.iters == 30 and err < 1e-9


def test_cpdl_with_randomized_topk(lib):
    import torch
    say("cpdl topk")
    p = synth.surface_pair(M=3000, N=3000, seed=6, beta=1.5, lam=2.0, w=0.2)
    X, Y = _f32(p.X), _f32(p.Y)
    K = 120
    r = lib.Registration(dev(X, torch.float32), dev(Y, torch.float32), precision="fp32",
                         method="cpdl", eig_mode="topk", K=K, beta=p.beta, lam=p.lam, w=p.w,
                         tol=0.0, max_iter=15)
    r.prepare()
    U, lam = (host(t) for t in r.export_eig())
    ref = cpd64.register(X, Y, p.beta, p.lam, p.w, "cpdl", eig=(U, lam), iters=15)
    out = r.register()
    err = cpd64.rel_rms(host(out.Xt), ref.Xt)
    say("rel_rms", err)
    assert err < 1e-5
