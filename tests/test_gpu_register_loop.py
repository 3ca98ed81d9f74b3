"""The register loop and single steps on one handle.

cpd_register enqueues iterations in batches of eight, keeps two batches in
flight and stops on the convergence flag the sigma^2 kernel sets on the
device; the launches still queued after convergence return at once.
cpd_step runs one ungated iteration.  Checked here: runs from the same start
state on one handle agree bit for bit whatever the previous call left
queued; a capped run stops at its cap when the cap is not a multiple of the
batch; a capped registration equals the same number of single steps; steps
after a converged registration still iterate."""
import pytest

import synth
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu


def _pair():
    return synth.surface_pair(M=2000, N=2200, seed=41, beta=2.0, lam=3.0, w=0.1,
                              outlier_frac=0.05)


def _reg(lib, X, Y, p, precision, **kw):
    return lib.Registration(X, Y, precision=precision, beta=p.beta, lam=p.lam, w=p.w,
                            eig_mode="topk", K=100, seed=3, **kw)


@pytest.mark.parametrize("precision", ["fp32", "bf16x"])
def test_repeated_register_calls_agree(lib, precision):
    import torch
    p = _pair()
    X, Y = dev(p.X, torch.float32), dev(p.Y, torch.float32)
    r = _reg(lib, X, Y, p, precision, tol=1e-8, max_iter=1000)
    X0, _, s20 = r.state()
    r.prepare()
    outs = []
    for _ in range(3):
        r.set_state(X0, s20)
        outs.append(r.register())
    a = outs[0]
    say(precision, "iters", [o.iters for o in outs], "sigma2", a.sigma2)
    assert a.converged and 8 < a.iters < 1000
    for b in outs[1:]:
        assert b.iters == a.iters and b.converged and b.sigma2 == a.sigma2
        assert torch.equal(b.Xt, a.Xt) and torch.equal(b.W, a.W)
    info = lib.cpd_step(r.h)  # ungated: iterates past the converged state
    assert info.iter == a.iters + 1
    r.close()


@pytest.mark.parametrize("cap", [5, 13, 21])
def test_capped_register_equals_single_steps(lib, cap):
    import torch
    p = _pair()
    X, Y = dev(p.X, torch.float32), dev(p.Y, torch.float32)
    r = _reg(lib, X, Y, p, "fp32", tol=0.0, max_iter=cap)
    X0, _, s20 = r.state()
    r.prepare()
    out = r.register()
    assert out.iters == cap and not out.converged
    r.set_state(X0, s20)
    for k in range(cap):
        info = lib.cpd_step(r.h)
    Xs, Ws, s2s = r.state()
    say("cap", cap, "sigma2", out.sigma2, s2s)
    assert info.iter == 2 * cap  # set_state keeps the iteration count
    assert s2s == out.sigma2
    assert torch.equal(Xs, out.Xt) and torch.equal(Ws, out.W)
    r.close()
