"""GPU parity of the original CPD comparator (eq. 21, FP64 blocked Cholesky)
against the FP64 oracle (scipy Cholesky), through the C ABI."""
import numpy as np
import pytest

import synth
from oracle import cpd64, eig64
from tests.gpu_util import dev, host, say, torch_dtype

pytestmark = pytest.mark.gpu


def _f32(a):
    return a.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("precision,M,N", [("fp64", 700, 650), ("fp64", 128, 300),
                                           ("fp32", 1000, 1100), ("fp64", 1, 5)])
def test_one_original_step(lib, precision, M, N):
    say("original one step", precision, M, N)
    p = synth.sphere_pair(M=M, N=N, seed=M)
    X, Y = (p.X, p.Y) if precision == "fp64" else (_f32(p.X), _f32(p.Y))
    rng = np.random.default_rng(3)
    Xt = X + 0.03 * rng.normal(size=X.shape)
    if precision == "fp32":
        Xt = _f32(Xt)
    s2 = 0.05
    dt = torch_dtype(precision)
    r = lib.Registration(dev(X, dt), dev(Y, dt), precision=precision, method="original",
                         beta=p.beta, lam=p.lam, w=p.w)
    r.prepare()
    r.set_state(dev(Xt, dt), s2)
    info = r.step()
    Xg, Wg, s2g = r.state()
    es = cpd64.estep(Xt, Y, s2, p.w)
    Phi = eig64.gram(X, p.beta)
    W, Xn = cpd64.cpd_mstep(X, es.P1, es.PY, Phi, p.lam, s2)
    s2n = cpd64.sigma2_cpd(Xt, Y, s2, es, Xn)
    tol = 1e-10 if precision == "fp64" else 1e-5
    err = cpd64.rel_rms(host(Xg), Xn)
    say("rel_rms", err)
    assert err < tol
    assert s2g == pytest.approx(s2n, rel=10 * tol)


def test_original_small500_fifty_iterations(lib):
    import torch
    say("original small500 x50")
    p = synth.workload("small500")
    ref = cpd64.register(p.X, p.Y, p.beta, p.lam, p.w, "cpd", iters=50)
    r = lib.Registration(dev(p.X, torch.float64), dev(p.Y, torch.float64), precision="fp64",
                         method="original", beta=p.beta, lam=p.lam, w=p.w, tol=0.0, max_iter=50)
    out = r.prepare().register()
    err = cpd64.rel_rms(host(out.Xt), ref.Xt)
    say("rel_rms", err)
    assert out.iters == 50 and err < 1e-9


def test_breakdown_is_reported(lib):
    """Duplicate model points make Phi singular; with a vanishing lambda
    sigma^2 / P1 shift the factorisation cannot proceed and the call must
    return CPD_E_NUMERIC rather than garbage."""
    import torch
    say("cholesky breakdown")
    X = np.zeros((200, 3))
    X[100:] = 1e-9          # two clusters of identical points: rank-2 Phi
    Y = np.random.default_rng(0).normal(size=(150, 3))
    r = lib.Registration(dev(X, torch.float64), dev(Y, torch.float64), precision="fp64",
                         method="original", beta=1.0, lam=1e-300, w=0.1)
    r.prepare()
    with pytest.raises(lib.FastCPDError) as e:
        r.step()
    assert e.value.status == lib.CPD_E_NUMERIC
