"""Where a warm start leaves sigma^2: the start of every run is set by that
run's own arguments, never by what an earlier run on the same handle left.

* Single handle: cpd_register with W0 starts from Xt = X + Phi W0 with the
  closed-form sigma^2 at that Xt (or sigma2_init when given), so running it
  twice on one handle gives the same result, and that result is the oracle's
  EM loop started from the same W0 (eq. 9-11 for Xt_0, eq. 17-18 per step).
* Batched handle: a warm-start run followed by a run from W = 0 gives exactly
  what a fresh batch gives from W = 0 (the second run restarts at the data's
  sigma^2_0, not at the warm start's)."""
import numpy as np
import pytest

import synth
from oracle import cpd64, eig64
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


def _f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("given", [0.0, 0.05])
def test_single_handle_warm_start_twice_matches_oracle(lib, given):
    import torch
    p = synth.sphere_pair(M=300, N=280, seed=21, coef=0.05)
    X, Y = _f32(p.X), _f32(p.Y)
    W0 = _f32(np.random.default_rng(5).normal(0.0, 0.02, X.shape))
    iters = 20
    say("warm reset single, sigma2_init", given)
    r = lib.Registration(dev(X, torch.float32), dev(Y, torch.float32), precision="fp32",
                         beta=p.beta, lam=p.lam, w=p.w, eig_mode="full", tol=0.0,
                         max_iter=iters, sigma2_init=given)
    r.prepare()
    a = r.register(W0=dev(W0, torch.float32))
    b = r.register(W0=dev(W0, torch.float32))
    U, lam = (host(t) for t in r.export_eig())
    r.close()
    assert a.iters == b.iters == iters
    assert torch.equal(a.Xt, b.Xt) and a.sigma2 == b.sigma2
    ref = cpd64.register(X, Y, p.beta, p.lam, p.w, "fast", eig=(U, lam), W0=W0,
                         Phi=eig64.gram(X, p.beta), sigma2_0=given or None, iters=iters)
    err = cpd64.rel_rms(host(a.Xt), ref.Xt)
    say("rel_rms vs oracle", err, "sigma2", a.sigma2, ref.sigma2)
    assert err < 1e-5
    assert abs(a.sigma2 - ref.sigma2) < 1e-5 * ref.sigma2


def test_batch_zero_start_after_warm_start_matches_fresh_batch(lib):
    import torch
    pairs = [synth.surface_pair(M=m, N=n, seed=40 + i, beta=2.0, lam=3.0, w=0.1)
             for i, (m, n) in enumerate([(700, 650), (520, 900), (1100, 800)])]
    Xs = [dev(_f32(q.X), torch.float32) for q in pairs]
    Ys = [dev(_f32(q.Y), torch.float32) for q in pairs]
    kw = dict(beta=[q.beta for q in pairs], lam=[q.lam for q in pairs], w=0.1,
              eig_mode="full", tol=1e-8, max_iter=300)
    W0 = torch.cat([0.01 * torch.randn(x.shape[0], 3, generator=torch.Generator().manual_seed(i))
                    for i, x in enumerate(Xs)]).float().cuda().contiguous()
    say("warm reset batch: warm arm then zero arm")
    br = lib.BatchRegistration(Xs, Ys, **kw).prepare(tune=False)
    br.register(W0=W0)
    Xa, ra = br.register()
    br.close()
    fresh = lib.BatchRegistration(Xs, Ys, **kw).prepare(tune=False)
    Xb, rb = fresh.register()
    fresh.close()
    for i in range(len(pairs)):
        say("instance", i, "iters", ra[i].iters, rb[i].iters, "sigma2", ra[i].sigma2, rb[i].sigma2)
        assert ra[i].iters == rb[i].iters and ra[i].sigma2 == rb[i].sigma2
        assert torch.equal(Xa[i], Xb[i])
