"""The internal spatial order and the E-step's far-tile culling.

* Culling is exact: a registration with culling and one without, on the same
  (sorted) handle configuration, give bit-identical points and iteration
  counts, in FP32 and BF16X.
* Culling is active: at a small sigma^2 on 20 000 points the E-step passes
  with culling take clearly less time than the passes without it (so the
  test fails if no tile is skipped), with bit-identical E-step outputs.
* The order is invisible: sorted and unsorted handles agree, step by step
  and on the standalone E-step outputs (FP32: each side is within 1e-5 of
  the exact trajectory, so they are held to 2e-5 of each other)."""
import numpy as np
import pytest

import synth
from oracle import cpd64
from tests.gpu_util import dev, host, say, torch_dtype

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "bf16x"])
def test_culling_is_bit_exact(lib, precision):
    import torch
    p = synth.surface_pair(M=6000, N=5000, seed=11, beta=2.0, lam=3.0, w=0.7, outlier_frac=0.05)
    X, Y = dev(p.X, torch.float32), dev(p.Y, torch.float32)
    out = {}
    for cull in (False, True):
        say("cull", precision, cull)
        r = lib.Registration(X, Y, precision=precision, beta=2.0, lam=3.0, w=0.7,
                             eig_mode="topk", K=100, seed=3, tol=1e-8, max_iter=400, cull=cull)
        r.prepare()
        res = r.register()
        out[cull] = res
        r.close()
    a, b = out[False], out[True]
    say("iters", a.iters, b.iters, "sigma2", a.sigma2)
    assert a.iters == b.iters and a.sigma2 == b.sigma2
    assert torch.equal(a.Xt, b.Xt) and torch.equal(a.W, b.W)


@pytest.mark.parametrize("precision", ["fp32", "bf16x"])
def test_culling_is_active_at_small_sigma2(lib, precision):
    import torch
    p = synth.surface_pair(M=20000, N=20000, seed=12, beta=2.0, lam=3.0, w=0.7, outlier_frac=0.05)
    X, Y = dev(p.X, torch.float32), dev(p.Y, torch.float32)
    Xs = dev(p.Y_hat, torch.float32)  # the true positions: a registered state
    out = {}
    for cull in (False, True):
        say("active", precision, cull)
        r = lib.Registration(X, Y, precision=precision, beta=2.0, lam=3.0, w=0.7,
                             eig_mode="import", K=1, cull=cull)
        # any valid eigenpair will do: only the E-step is timed and compared
        U = torch.full((p.M, 1), p.M ** -0.5, dtype=torch.float64, device="cuda")
        r.prepare(U=U, lam=torch.ones(1, dtype=torch.float64, device="cuda"))
        r.set_state(Xs, 1e-3)
        g = r.estep()
        r.set_state(Xs, 1e-3)
        kern = r.time_kernels(reps=5)
        out[cull] = ({k: v.clone() for k, v in g.items()}, kern)
        r.close()
    (ga, ka), (gb, kb) = out[False], out[True]
    say("passA ms", ka["passA"], kb["passA"], "passB ms", ka["passB"], kb["passB"])
    for k in ga:
        assert torch.equal(ga[k], gb[k]), k
    assert kb["passA"] < 0.85 * ka["passA"] and kb["passB"] < 0.85 * ka["passB"]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-5)])
def test_internal_order_is_invisible(lib, precision, tol):
    p = synth.workload("small500")
    dt = torch_dtype(precision)
    X, Y = dev(p.X, dt), dev(p.Y, dt)
    runs = {}
    for sort in (False, True):
        say("order", precision, sort)
        r = lib.Registration(X, Y, precision=precision, beta=p.beta, lam=p.lam, w=p.w,
                             eig_mode="full", tol=0.0, max_iter=20, sort=sort)
        r.prepare()
        res = r.register()
        g = r.estep()
        U, lam = r.export_eig()
        runs[sort] = (host(res.Xt), {k: host(v) for k, v in g.items()}, host(U), host(lam))
        r.close()
    (xa, ga, Ua, la), (xb, gb, Ub, lb) = runs[False], runs[True]
    assert cpd64.rel_rms(xb, xa) < tol
    np.testing.assert_allclose(gb["logd"], ga["logd"], rtol=0, atol=50 * tol * np.abs(ga["logd"]).max())
    np.testing.assert_allclose(gb["P1"], ga["P1"], rtol=100 * tol, atol=1e-30)
    assert cpd64.rel_rms(gb["Yt"], ga["Yt"]) < 10 * tol
    # exported eigenvectors are in the caller's row order: U Lam U^T is the
    # same Gram matrix (a row permutation would scramble it)
    np.testing.assert_allclose(lb, la, rtol=1e-9, atol=1e-12 * la.max())
    Ga, Gb = (Ua * la) @ Ua.T, (Ub * lb) @ Ub.T
    assert np.abs(Ga - Gb).max() < 1e-10 * la.max()
