"""Write the stored expected values under tests/golden/ from the FP64 oracle.

    python tests/golden/make_golden.py [name ...]      (default: every fixture)

Calls nothing but oracle/ and synth/.  Each .npz holds the oracle's outputs
plus a `meta` JSON string naming the workload, its sizes and parameters, the
oracle calls and the seeds, so a test can rebuild the exact inputs from synth
and compare.  Inputs that a GPU test feeds in float32 are rounded to float32
here first, so the oracle sees the very values the device sees.

Fixtures (one function each below):
  affine4000   the scaling study's protocol (Section IV-B, Table IV): CPD,
               CPD-L, Fast CPD (full eigendecomposition) and Fast CPD-L on
               an affine pair, M = N = 4000, K = 0.1 M, 50 iterations.
  surface10k   cfg2: Fast CPD with all eigenpairs (eq. 17) and original CPD
               (eq. 21) on the 10k surface pair, to |dsigma^2| < 1e-8.
  surface50k   the 50k surface pair: top-300 eigenpairs from a stored-seed
               test matrix (eq. 19), their projections of three probes, and
               20 Fast CPD iterations (eq. 20) from the closed-form sigma^2_0.
  surface20k_w02  the 50k recipe at M = N = 20 000 (w = 0.2, 20% outliers):
               the sigma^2 and RMSE traces over 250 Fast CPD iterations.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import cpd64, eig64  # noqa: E402


def _f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def _log(*a):
    print(f"[{time.strftime('%H:%M:%S')}]", *a, flush=True)


def _save(name, meta, **arrays):
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, meta=np.array(json.dumps(meta, sort_keys=True)), **arrays)
    _log("wrote", path, f"{os.path.getsize(path) / 1024:.0f} KiB")


def _trace(r):
    return np.array([t[0] for t in r.trace])


def affine4000():
    M, iters, seed_omega = 4000, 50, 0
    p = synth.affine_pair(M, seed=0)
    X, Y = _f32(p.X), _f32(p.Y)
    K, over, q = M // 10, 20, 2
    Om = synth.gaussian_matrix(M, K + over, seed_omega)
    Phi = eig64.gram(X, p.beta)
    t = time.time()
    full = eig64.eig_full(Phi)
    topk = eig64.eig_topk(X, p.beta, K, Om, q)
    _log("affine4000 eig", f"{time.time() - t:.1f}s")
    out, meta_runs = {}, {}
    runs = (("cpd", dict(method="cpd", Phi=Phi)),
            ("cpdl", dict(method="cpdl", eig=topk)),
            ("fast_full", dict(method="fast", eig=full)),
            ("fast_topk", dict(method="fast", eig=topk)))
    for name, kw in runs:
        t = time.time()
        r = cpd64.register(X, Y, p.beta, p.lam, p.w, iters=iters, **kw)
        _log("affine4000", name, f"{time.time() - t:.1f}s", "sigma2", r.sigma2)
        out[f"Xt_{name}"] = r.Xt
        out[f"sigma2_{name}"] = _trace(r)
        meta_runs[name] = {"method": kw["method"],
                           "eig": {"cpdl": "topk", "fast_topk": "topk",
                                   "fast_full": "full"}.get(name)}
    out["lam_topk"] = topk[1]
    meta = {"workload": "synth.affine_pair(4000, seed=0), inputs rounded to float32",
            "M": M, "N": M, "beta": p.beta, "lam": p.lam, "w": p.w, "iters": iters,
            "K": K, "oversample": over, "power_iters": q,
            "omega": f"synth.gaussian_matrix(M, K + oversample, seed={seed_omega})",
            "runs": meta_runs,
            "oracle": "cpd64.register(X, Y, beta, lam, w, method, iters=50) with "
                      "eig64.eig_full(gram) or eig64.eig_topk(X, beta, K, omega, q)"}
    _save("affine4000", meta, **out)


def surface10k():
    p = synth.workload("surface10k")
    X, Y = _f32(p.X), _f32(p.Y)
    tol, cap = 1e-8, 1000
    Phi = eig64.gram(X, p.beta)
    t = time.time()
    full = eig64.eig_full(Phi)
    _log("surface10k eigh", f"{time.time() - t:.1f}s")
    out = {"lam_full": full[1]}
    for name, kw in (("fast_full", dict(method="fast", eig=full)),
                     ("cpd", dict(method="cpd", Phi=Phi))):
        t = time.time()
        r = cpd64.register(X, Y, p.beta, p.lam, p.w, tol=tol, max_iter=cap, **kw)
        _log("surface10k", name, f"{time.time() - t:.1f}s", "iters", r.iters,
             "converged", r.converged, "sigma2", r.sigma2)
        out[f"Xt_{name}"] = r.Xt
        out[f"sigma2_{name}"] = _trace(r)
        out[f"iters_{name}"] = np.array(r.iters)
        out[f"converged_{name}"] = np.array(r.converged)
        out[f"rmse_{name}"] = np.array(cpd64.rmse(r.Xt, p.Y_hat))
    meta = {"workload": "synth.workload('surface10k'), inputs rounded to float32",
            "M": p.M, "N": p.N, "beta": p.beta, "lam": p.lam, "w": p.w, "tol": tol,
            "max_iter": cap,
            "oracle": "cpd64.register(X, Y, beta, lam, w, 'fast', eig=eig64.eig_full(gram)) "
                      "and cpd64.register(..., 'cpd', Phi=gram), tol=1e-8"}
    _save("surface10k", meta, **out)


def surface50k():
    p = synth.workload("surface50k")
    X, Y = _f32(p.X), _f32(p.Y)
    M = p.M
    K, over, q, seed_omega, iters = 300, 20, 2, 0, 20
    Om = synth.gaussian_matrix(M, K + over, seed_omega)
    t = time.time()
    U, lam = eig64.eig_topk(X, p.beta, K, Om, q)
    del Om
    _log("surface50k eig_topk", f"{time.time() - t:.1f}s", "lam_1", lam[0], "lam_K", lam[-1])
    rows = np.sort(np.random.default_rng(5).choice(M, 2048, replace=False))
    # the rank-K Gram Phi~ = U Lam U^T (eq. 19) and the Fast M-step's operator
    # U diag(lam / (lam + lambda s2)) U^T (eq. 20) at s2 = 1e-3, applied to
    # three probes: invariant to the sign and the basis of the eigenvectors
    lp = np.maximum(lam, 0.0)
    gram_probe, mstep_probe = [], []
    for j in range(3):
        T = U.T @ synth.gaussian_matrix(M, 3, 100 + j)
        gram_probe.append((U[rows] @ (lp[:, None] * T)))
        mstep_probe.append((U[rows] @ ((lp / (lp + p.lam * 1e-3))[:, None] * T)))
    t = time.time()
    r = cpd64.register(X, Y, p.beta, p.lam, p.w, "fast", eig=(U, lam), iters=iters)
    _log("surface50k", iters, "iterations", f"{time.time() - t:.1f}s", "sigma2", r.sigma2)
    meta = {"workload": "synth.workload('surface50k'), inputs rounded to float32",
            "M": M, "N": p.N, "beta": p.beta, "lam": p.lam, "w": p.w, "K": K,
            "oversample": over, "power_iters": q,
            "omega": f"synth.gaussian_matrix(M, K + oversample, seed={seed_omega})",
            "probes": "R_j = synth.gaussian_matrix(M, 3, seed=100 + j), j = 0, 1, 2",
            "probe_rows": "np.random.default_rng(5).choice(M, 2048, replace=False), sorted",
            "gram_probe": "(U diag(lam+) U^T R_j)[rows]",
            "mstep_probe": "(U diag(lam+ / (lam+ + lambda 1e-3)) U^T R_j)[rows]",
            "iters": iters,
            "oracle": "U, lam = eig64.eig_topk(X, beta, K, omega, q); the probes; "
                      "cpd64.register(X, Y, beta, lam, w, 'fast', eig=(U, lam), iters=20) "
                      "from the closed-form sigma^2_0"}
    _save("surface50k", meta, lam=lam, probe_rows=rows, gram_probe=np.stack(gram_probe),
          mstep_probe=np.stack(mstep_probe), Xt=r.Xt.astype(np.float32), sigma2=_trace(r))


def surface20k_w02():
    M, iters = 20000, 250
    p = synth.workload("surface50k", M=M)
    K, over, q, seed_omega = 300, 20, 2, 0
    Om = synth.gaussian_matrix(M, K + over, seed_omega)
    t = time.time()
    U, lam = eig64.eig_topk(p.X, p.beta, K, Om, q)
    _log("surface20k eig_topk", f"{time.time() - t:.1f}s")
    X, Y = p.X, p.Y
    Xt = X.copy()
    s2 = cpd64.sigma2_init(Xt, Y)
    s2_0 = s2
    sig, err = [], []
    t = time.time()
    for k in range(iters):
        es = cpd64.estep(Xt, Y, s2, p.w)
        _, Xn = cpd64.fast_mstep(X, es.Yt, U, lam, p.lam, s2)
        s2 = max(cpd64.sigma2_fast(Xt, Y, s2, es, Xn), 1e-10 * s2_0)
        Xt = Xn
        sig.append(s2)
        err.append(cpd64.rmse(Xt, p.Y_hat))
        if (k + 1) % 10 == 0:
            _log("surface20k iteration", k + 1, "sigma2", s2, "rmse", err[-1],
                 f"{(time.time() - t) / (k + 1):.1f}s/it")
    meta = {"workload": "synth.workload('surface50k', M=20000) (float64 inputs)",
            "M": M, "N": p.N, "beta": p.beta, "lam": p.lam, "w": p.w, "K": K,
            "oversample": over, "power_iters": q,
            "omega": f"synth.gaussian_matrix(M, K + oversample, seed={seed_omega})",
            "iters": iters,
            "oracle": "eig64.eig_topk; then per iteration cpd64.estep, cpd64.fast_mstep, "
                      "cpd64.sigma2_fast (floor 1e-10 sigma^2_0), cpd64.rmse against Y_hat"}
    _save("surface20k_w02", meta, sigma2=np.array(sig), rmse=np.array(err),
          Xt=Xt.astype(np.float32), lam=lam)


FIXTURES = {"affine4000": affine4000, "surface10k": surface10k, "surface50k": surface50k,
            "surface20k_w02": surface20k_w02}

if __name__ == "__main__":
    names = sys.argv[1:] or list(FIXTURES)
    for n in names:
        _log("start", n)
        FIXTURES[n]()
