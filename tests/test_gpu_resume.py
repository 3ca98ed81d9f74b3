"""Determinism and resumption.

Every reduction on the GPU path is two-stage and fixed-order (no float
atomics), so two runs of the same registration are bitwise identical: that
is the race check.  The EM iteration's state is (Xt, sigma^2): W is
recomputed from Yt alone every iteration (eq. 17), so a registration split
into two runs, the second on a fresh handle given the first's eigenpairs
(cpd_eig_export / CPD_EIG_IMPORT) and state (cpd_set_state), continues the
same iteration."""
import numpy as np
import pytest

import synth
from oracle import cpd64
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


def _pair(M=3000, N=3200, seed=31):
    return synth.surface_pair(M=M, N=N, seed=seed, beta=2.0, lam=3.0, w=0.2, outlier_frac=0.1)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x"])
def test_two_runs_are_bitwise_identical(lib, precision):
    import torch
    p = _pair()
    dt = torch.float64 if precision == "fp64" else torch.float32
    X, Y = dev(p.X, dt), dev(p.Y, dt)
    outs = []
    for run in range(2):
        r = lib.Registration(X, Y, precision=precision, beta=p.beta, lam=p.lam, w=p.w,
                             eig_mode="topk", K=150, seed=9, tol=0.0, max_iter=60)
        r.prepare()
        outs.append(r.register())
        r.close()
    a, b = outs
    say(precision, "sigma2", a.sigma2, b.sigma2)
    assert a.iters == b.iters == 60 and a.sigma2 == b.sigma2
    assert torch.equal(a.Xt, b.Xt) and torch.equal(a.W, b.W)


def test_two_batched_runs_are_bitwise_identical(lib):
    import torch
    pairs = [synth.surface_pair(M=m, N=n, seed=50 + i, beta=2.0, lam=3.0, w=0.1,
                                outlier_frac=0.05)
             for i, (m, n) in enumerate([(700, 900), (1500, 1200), (2600, 2500), (400, 380)])]
    Xs = [dev(q.X, torch.float32) for q in pairs]
    Ys = [dev(q.Y, torch.float32) for q in pairs]
    outs = []
    for run in range(2):
        br = lib.BatchRegistration(Xs, Ys, beta=[q.beta for q in pairs],
                                   lam=[q.lam for q in pairs], w=0.1, eig_mode="full",
                                   tol=0.0, max_iter=40)
        Xt, res = br.prepare(tune=False).register()
        outs.append(([x.clone() for x in Xt], [r.sigma2 for r in res]))
        br.close()
    (x0, s0), (x1, s1) = outs
    assert s0 == s1
    assert all(torch.equal(a, b) for a, b in zip(x0, x1))


@pytest.mark.parametrize("precision,sort", [("fp64", False), ("fp32", False), ("bf16x", False),
                                            ("fp64", True)])
def test_resume_on_a_fresh_handle_continues_the_iteration(lib, precision, sort):
    """40 steps on one handle against 15 steps, then export of (U, lam) and
    (Xt, sigma^2), then 25 steps on a fresh handle that imports both.  In
    the caller's frame (sort = False) the two paths are bitwise identical;
    with the internal spatial order the state passes through the caller's
    frame once (points shifted back and forth in double, stored in the
    working precision), so FP64 agrees to 1e-12."""
    import torch
    p = _pair(seed=32)
    dt = torch.float64 if precision == "fp64" else torch.float32
    X, Y = dev(p.X, dt), dev(p.Y, dt)
    kw = dict(precision=precision, beta=p.beta, lam=p.lam, w=p.w, tol=0.0, max_iter=100,
              sort=sort)
    ref = lib.Registration(X, Y, eig_mode="topk", K=120, seed=4, **kw)
    ref.prepare()
    for _ in range(40):
        ref.step()
    Xref, _, s2ref = ref.state()
    a = lib.Registration(X, Y, eig_mode="topk", K=120, seed=4, **kw)
    a.prepare()
    for _ in range(15):
        a.step()
    Xa, _, s2a = a.state()
    U, lam = a.export_eig()
    b = lib.Registration(X, Y, eig_mode="import", K=U.shape[1], **kw)
    b.prepare(U=U, lam=lam)
    b.set_state(Xa, s2a)
    for _ in range(25):
        b.step()
    Xb, _, s2b = b.state()
    err = cpd64.rel_rms(host(Xb), host(Xref))
    say(precision, "sort", sort, "resumed vs straight: rel_rms", err, "sigma2", s2b, s2ref)
    if not sort:
        assert torch.equal(Xb, Xref) and s2b == s2ref
    else:
        assert err < 1e-12 and s2b == pytest.approx(s2ref, rel=1e-12)
    for h in (ref, a, b):
        h.close()
