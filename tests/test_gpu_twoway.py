"""Two-way registration (Section IV-A) on the GPU: the nearest-neighbour
matches and the matched solve against the oracle (FP64, exact eigenpairs of
the dense solver), and the whole scheme on a scene with a missing cap."""
import numpy as np
import pytest

import synth
from oracle import cpd64, eig64
from tests.gpu_util import dev, host, say, torch_dtype

pytestmark = pytest.mark.gpu


def _occluded(seed=4, M=300):
    # the field keeps the size it has at 300 points (coefficients ~ 1/sqrt(M))
    p = synth.sphere_pair(M=M, N=M, seed=seed, coef=0.03 * np.sqrt(300.0 / M), outlier_frac=0.0)
    keep = p.Y[:, 2] < 0.35
    return p, np.ascontiguousarray(p.Y[keep])


@pytest.mark.parametrize("mutual", [True, False])
def test_matches_equal_brute_force(lib, mutual):
    import torch
    say("matches", mutual)
    rng = np.random.default_rng(5)
    X = rng.normal(size=(700, 3))
    Y = rng.normal(size=(530, 3))
    Xt = X + 0.05 * rng.normal(size=X.shape)
    r = lib.Registration(dev(X, torch.float64), dev(Y, torch.float64), precision="fp64",
                         eig_mode="import", K=1)
    r.set_state(dev(Xt, torch.float64), 0.1)
    got = host(r.matches(mutual_only=mutual)).astype(np.int64)
    ref = cpd64.mutual_matches(Y, Xt) if mutual else cpd64.nearest(Y, Xt)
    assert np.array_equal(got, ref)


def test_solve_matches_equals_the_matched_mstep(lib):
    import torch
    say("solve matches")
    p, Y = _occluded()
    rng = np.random.default_rng(6)
    match = np.where(rng.random(p.M) < 0.5, rng.integers(0, Y.shape[0], p.M), -1)
    s2 = 0.02
    r = lib.Registration(dev(p.X, torch.float64), dev(Y, torch.float64), precision="fp64",
                         beta=p.beta, lam=p.lam, w=0.1, eig_mode="full")
    r.prepare()
    Xt, W = r.solve_matches(dev(match, torch.int32), s2)
    ref_W, ref_Xt = cpd64.matched_mstep(p.X, Y, match, eig64.gram(p.X, p.beta), p.lam, s2)
    err = cpd64.rel_rms(host(Xt), ref_Xt)
    say("rel_rms", err)
    assert err < 1e-9


def test_two_way_end_to_end_fp64(lib):
    say("two-way fp64")
    import torch
    p, Y = _occluded()
    kw = dict(beta=p.beta, lam=p.lam, w=0.1, eig_mode="full", tol=0.0, max_iter=60,
              precision="fp64")
    Xt, W, match, first = lib.register_two_way(dev(p.X, torch.float64), dev(Y, torch.float64), **kw)
    ref_Xt, ref_W, ref_match, ref_first = cpd64.register_two_way(p.X, Y, p.beta, p.lam, 0.1,
                                                                 iters=60)
    m = host(match).astype(np.int64)
    say("matches", (m >= 0).sum(), (ref_match >= 0).sum(), "differ", int((m != ref_match).sum()))
    assert (m != ref_match).sum() <= 1
    err = cpd64.rel_rms(host(Xt), ref_Xt)
    e_two, e_ref = cpd64.rmse(host(Xt), p.Y_hat), cpd64.rmse(ref_Xt, p.Y_hat)
    say("rel_rms", err, "rmse", e_two, e_ref)
    if (m == ref_match).all():
        assert err < 1e-8
    assert e_two == pytest.approx(e_ref, rel=1e-3)


def test_two_way_beats_direct_registration_fp32(lib):
    """2000 points, the scene's top cap missing (35% of the points): the FP64
    oracle gives RMSE 0.671 direct and 0.481 two-way after 60 iterations."""
    say("two-way fp32 gain")
    import torch
    p, Y = _occluded(seed=8, M=2000)
    kw = dict(beta=p.beta, lam=p.lam, w=0.1, eig_mode="full", tol=0.0, max_iter=60)
    X32, Y32 = dev(p.X, torch.float32), dev(Y, torch.float32)
    Xt, W, match, first = lib.register_two_way(X32, Y32, **kw)
    d = lib.Registration(X32, Y32, **kw)
    direct = d.prepare().register()
    d.close()
    e_two, e_dir = cpd64.rmse(host(Xt), p.Y_hat), cpd64.rmse(host(direct.Xt), p.Y_hat)
    say("rmse two-way", e_two, "direct", e_dir, "matches", int((host(match) >= 0).sum()))
    assert e_two < 0.85 * e_dir
