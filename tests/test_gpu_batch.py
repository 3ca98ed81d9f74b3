"""Batched registration (work-list kernels over all instances, one HIP graph
per iteration) against the FP64 oracle and the single-instance path."""
import numpy as np
import pytest

import synth
from oracle import cpd64, eig64
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


def _f32(a):
    return a.astype(np.float32).astype(np.float64)


def _instances(B, lo, hi, seed0):
    pairs = []
    for i in range(B):
        rng = np.random.default_rng(seed0 + i)
        M, N = int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))
        beta, lam = float(rng.uniform(1.0, 3.0)), float(rng.uniform(1.0, 5.0))
        pairs.append(synth.surface_pair(M=M, N=N, seed=seed0 + i, beta=beta, lam=lam, w=0.1,
                                        outlier_frac=0.05))
    return pairs


def test_batch_matches_oracle_per_instance(lib):
    """10 instances of 150..1800 points (dense FULL eigen-prep below 1025
    points with K = M, some K % 4 != 0, randomized above): every plan the
    tuner can choose (4 split lengths x 2 E-step tiles) and the tuned one
    give the oracle's 15 iterations within 1e-5."""
    import torch
    pairs = _instances(10, 150, 1800, 500)
    say("batch vs oracle", [(p.M, p.N) for p in pairs])
    Xs = [dev(_f32(p.X), torch.float32) for p in pairs]
    Ys = [dev(_f32(p.Y), torch.float32) for p in pairs]
    refs = []
    for p in pairs:
        X, Y = _f32(p.X), _f32(p.Y)
        refs.append(cpd64.register(X, Y, p.beta, p.lam, p.w, "fast",
                                   eig=eig64.eig_full(eig64.gram(X, p.beta)), iters=15).Xt)
    br = lib.BatchRegistration(Xs, Ys, beta=[p.beta for p in pairs], lam=[p.lam for p in pairs],
                               w=0.1, eig_mode="full", tol=0.0, max_iter=15)
    plans = [None] + list(range(8))
    for cand in plans:
        if cand is None:
            br.prepare(tune=True)
        else:
            br.prepare(candidate=cand)
        info = br.info()
        say("plan", cand, "chunk", info["chunk"], "tile", info["tile"], "K", info["K"])
        if cand is not None:
            assert (info["chunk"], info["tile"]) == lib.BatchRegistration.candidates()[cand]
        else:
            assert all(v > 0 for v in info["tune_ms"].values())
        Xt, res = br.register()
        for p, x, r, ref in zip(pairs, Xt, res, refs):
            err = cpd64.rel_rms(host(x), ref)
            assert r.iters == 15 and err < 1e-5, (cand, p.M, p.N, err)
        assert any(k % 4 for k in info["K"]) and any(k % 4 == 0 for k in info["K"])
    br.close()


def test_batch_instances_stop_independently(lib):
    """With a tolerance, each instance stops at its own iteration; results
    agree with single-instance registrations of the same pairs."""
    import torch
    pairs = _instances(6, 300, 1200, 900)
    Xs = [dev(_f32(p.X), torch.float32) for p in pairs]
    Ys = [dev(_f32(p.Y), torch.float32) for p in pairs]
    kw = dict(w=0.1, eig_mode="full", tol=1e-6, max_iter=300)
    br = lib.BatchRegistration(Xs, Ys, beta=[p.beta for p in pairs],
                               lam=[p.lam for p in pairs], **kw)
    Xt, res = br.prepare(tune=False).register()
    iters = [r.iters for r in res]
    say("batch iterations", iters)
    for p, x, r, X, Y in zip(pairs, Xt, res, Xs, Ys):
        single = lib.Registration(X, Y, precision="fp32", beta=p.beta, lam=p.lam, **kw)
        out = single.prepare().register()
        assert r.converged and out.converged
        assert abs(r.iters - out.iters) <= 1
        if r.iters == out.iters:
            assert cpd64.rel_rms(host(x), host(out.Xt)) < 1e-5
    assert len(set(iters)) > 1


def test_batch_eigen_prep_in_several_waves_matches_single_handles(lib):
    """70 instances (three waves of the prepare's host threads, whose Jacobi
    solves run grouped by size class: dense solves below 1025 points, the
    256-column Rayleigh-Ritz solves above) give every instance the eigenpairs
    a single handle computes: the same K, eigenvalues within 1e-12 lam_1 and
    the same registration after 10 iterations (1e-5).  An unknown tuning
    code is refused."""
    import torch
    pairs = _instances(70, 200, 2600, 4000)
    Xs = [dev(_f32(p.X), torch.float32) for p in pairs]
    Ys = [dev(_f32(p.Y), torch.float32) for p in pairs]
    kw = dict(w=0.1, eig_mode="full", tol=0.0, max_iter=10)
    br = lib.BatchRegistration(Xs, Ys, beta=[p.beta for p in pairs],
                               lam=[p.lam for p in pairs], **kw)
    with pytest.raises(lib.FastCPDError):
        br.prepare(candidate=8)
    br.prepare(tune=False)
    K = br.info()["K"]
    Xt, res = br.register()
    br.close()
    dense = sum(p.M <= 1024 for p in pairs)
    say("70 instances,", dense, "dense; K range", min(K), max(K))
    assert 0 < dense < 70
    for i, (p, x, X, Y) in enumerate(zip(pairs, Xt, Xs, Ys)):
        single = lib.Registration(X, Y, precision="fp32", beta=p.beta, lam=p.lam, **kw)
        single.prepare()
        assert single.K == K[i], (i, p.M, single.K, K[i])
        out = single.register()
        err = cpd64.rel_rms(host(x), host(out.Xt))
        assert err < 1e-5, (i, p.M, err)
        single.close()


def test_batch_tune_cache_reuses_plan(lib, tmp_path):
    """The first tuned batch stores its plan under the batch's key; a second
    batch of the same shape forces that plan untimed and gives the same
    result bitwise."""
    import json
    import torch
    pairs = _instances(5, 300, 900, 1300)
    Xs = [dev(_f32(p.X), torch.float32) for p in pairs]
    Ys = [dev(_f32(p.Y), torch.float32) for p in pairs]
    kw = dict(beta=[p.beta for p in pairs], lam=[p.lam for p in pairs], w=0.1,
              eig_mode="full", tol=0.0, max_iter=10)
    path = str(tmp_path / "tune.json")
    a = lib.BatchRegistration(Xs, Ys, **kw).prepare(tune=True, cache=path)
    ia = a.info()
    assert all(v > 0 for v in ia["tune_ms"].values())
    with open(path) as f:
        stored = json.load(f)["entries"]
    key = a.tune_key()
    say("tune cache", key, stored[key]["chunk"], stored[key]["tile"])
    assert key.startswith(torch.cuda.get_device_properties(0).gcnArchName + "|batch|")
    assert (stored[key]["chunk"], stored[key]["tile"]) == (ia["chunk"], ia["tile"])
    Xa, _ = a.register()
    b = lib.BatchRegistration(Xs, Ys, **kw).prepare(tune=True, cache=path)
    ib = b.info()
    assert all(v == 0 for v in ib["tune_ms"].values())
    assert (ib["chunk"], ib["tile"]) == (ia["chunk"], ia["tile"])
    Xb, _ = b.register()
    for x, y in zip(Xa, Xb):
        assert torch.equal(x, y)
    a.close()
    b.close()
