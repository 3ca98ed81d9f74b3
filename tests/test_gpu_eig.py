"""GPU eigen-prep (Section III, eq. 16 and eq. 19) against the FP64 oracle.

Eigenvectors are compared only through quantities invariant to their sign
and to rotations inside (near-)degenerate eigenspaces: eigenvalues, the
reconstruction U Lam U^T, orthonormality, and the registration they drive."""
import numpy as np
import pytest

import synth
from oracle import cpd64, eig64
from tests.gpu_util import dev, host, say, torch_dtype

pytestmark = pytest.mark.gpu


def _f32(a):
    return a.astype(np.float32).astype(np.float64)


def test_dense_jacobi_full_eig(lib):
    import torch
    say("dense jacobi M=500")
    p = synth.workload("small500")
    r = lib.Registration(dev(p.X, torch.float64), dev(p.Y, torch.float64), precision="fp64",
                         beta=p.beta, lam=p.lam, w=p.w, eig_mode="full")
    r.prepare()
    assert r.K == p.M
    U, lam = (host(t) for t in r.export_eig())
    Phi = eig64.gram(p.X, p.beta)
    lref = np.linalg.eigvalsh(Phi)[::-1]
    np.testing.assert_allclose(lam, lref, rtol=0, atol=1e-12 * lref[0])
    assert np.all(np.diff(lam) <= 0)
    assert np.linalg.norm(U @ np.diag(lam) @ U.T - Phi) / np.linalg.norm(Phi) < 1e-12 * np.sqrt(p.M)
    assert np.linalg.norm(U.T @ U - np.eye(p.M)) < 1e-12 * np.sqrt(p.M)


def test_small500_fp64_with_gpu_eig(lib):
    """The 500-point FP64 workload end to end: GPU eigendecomposition and
    50 EM iterations, against the oracle with scipy's eigh."""
    import torch
    say("small500 fp64 full eig x50")
    p = synth.workload("small500")
    ref = cpd64.register(p.X, p.Y, p.beta, p.lam, p.w, "fast",
                         eig=eig64.eig_full(eig64.gram(p.X, p.beta)), iters=50)
    r = lib.Registration(dev(p.X, torch.float64), dev(p.Y, torch.float64), precision="fp64",
                         beta=p.beta, lam=p.lam, w=p.w, eig_mode="full", tol=0.0, max_iter=50)
    out = r.prepare().register()
    err = cpd64.rel_rms(host(out.Xt), ref.Xt)
    say("rel_rms", err)
    # eigenpairs near round-off of lam_1 are fixed only to ~eps*lam_1 by any FP64
    # solver; through h = lam/(lam + lambda sigma^2) they move Xt by up to
    # ~eps*lam_1/(lambda sigma^2) ~ 4e-12 each (lam_1 ~ 394, lambda sigma^2 >= 0.012)
    assert out.iters == 50 and err < 1e-9


@pytest.mark.parametrize("given_omega", [True, False])
def test_randomized_topk(lib, given_omega):
    import torch
    say("randomized topk", given_omega)
    p = synth.surface_pair(M=3000, N=3000, seed=3, beta=1.5, lam=2.0, w=0.2)
    X = _f32(p.X)
    K, over, q = 100, 20, 2
    Om = synth.gaussian_matrix(p.M, K + over, seed=11)
    Uo, lo = eig64.eig_topk(X, p.beta, K, Om, power_iters=q)
    r = lib.Registration(dev(X, torch.float32), dev(_f32(p.Y), torch.float32), precision="fp32",
                         beta=p.beta, lam=p.lam, w=p.w, eig_mode="topk", K=K, oversample=over,
                         power_iters=q, seed=5, tol=0.0, max_iter=15)
    r.prepare(omega=dev(Om, torch.float64) if given_omega else None)
    U, lam = (host(t) for t in r.export_eig())
    # eigenvalues agree down to the FP64 round-off of the largest
    np.testing.assert_allclose(lam, lo, rtol=0, atol=1e-11 * lo[0])
    np.testing.assert_allclose(U.T @ U, np.eye(K), atol=1e-10)
    # residual |Phi u - lam u| on sampled rows (rows of Phi formed directly)
    rows = np.random.default_rng(0).choice(p.M, 50, replace=False)
    Phr = np.exp(-cpd64.sqdist(X[rows], X) / (2 * p.beta ** 2))
    big = lam > 1e-8 * lam[0]
    res = Phr @ U[:, big] - U[rows][:, big] * lam[big]
    assert np.abs(res).max() < 1e-9 * lam[0]
    ref = cpd64.register(X, _f32(p.Y), p.beta, p.lam, p.w, "fast", eig=(Uo, lo), iters=15)
    out = r.register()
    err = cpd64.rel_rms(host(out.Xt), ref.Xt)
    say("rel_rms", err)
    assert err < 1e-5


@pytest.mark.parametrize("M,K,over,precision", [(2503, 130, 20, "fp32"), (1507, 290, 30, "fp64")])
def test_randomized_topk_wide_tiles(lib, M, K, over, precision):
    """Widths served by 160-column output tiles (n = 150: ten padded columns;
    n = 320: two full tiles), ragged M, FP32 and FP64 point storage: every
    product with Phi splits its tiles over several blocks."""
    import torch
    say("randomized topk wide tiles", M, K + over, precision)
    p = synth.surface_pair(M=M, N=M, seed=8, beta=1.5, lam=2.0, w=0.2)
    X = _f32(p.X)
    q = 2
    Om = synth.gaussian_matrix(p.M, K + over, seed=12)
    Uo, lo = eig64.eig_topk(X, p.beta, K, Om, power_iters=q)
    dt = torch.float64 if precision == "fp64" else torch.float32
    r = lib.Registration(dev(X, dt), dev(_f32(p.Y), dt), precision=precision, beta=p.beta,
                         lam=p.lam, w=p.w, eig_mode="topk", K=K, oversample=over,
                         power_iters=q, seed=5, tol=0.0, max_iter=5)
    r.prepare(omega=dev(Om, torch.float64))
    U, lam = (host(t) for t in r.export_eig())
    err = np.abs(lam - lo).max() / lo[0]
    say("max |lam - lam_oracle| / lam_1", err)
    np.testing.assert_allclose(lam, lo, rtol=0, atol=1e-11 * lo[0])
    np.testing.assert_allclose(U.T @ U, np.eye(K), atol=1e-10)
    rows = np.random.default_rng(1).choice(p.M, 40, replace=False)
    Phr = np.exp(-cpd64.sqdist(X[rows], X) / (2 * p.beta ** 2))
    big = lam > 1e-8 * lam[0]
    res = Phr @ U[:, big] - U[rows][:, big] * lam[big]
    assert np.abs(res).max() < 1e-9 * lam[0]


def test_randomized_topk_wide_rayleigh_ritz(lib):
    """K + p = 1220 > 1024: the Rayleigh-Ritz matrix takes the block Jacobi
    (39 blocks of 32 columns, the last ragged, plus an empty one to pair
    with).  Eigenvalues against the oracle's eig_topk with the same test
    matrix, orthonormal vectors and residuals on sampled rows of Phi."""
    import torch
    say("randomized topk wide Rayleigh-Ritz")
    p = synth.surface_pair(M=2600, N=2600, seed=13, beta=1.5, lam=2.0, w=0.2)
    X = _f32(p.X)
    K, over, q = 1200, 20, 2
    Om = synth.gaussian_matrix(p.M, K + over, seed=14)
    Uo, lo = eig64.eig_topk(X, p.beta, K, Om, power_iters=q)
    r = lib.Registration(dev(X, torch.float64), dev(_f32(p.Y), torch.float64), precision="fp64",
                         beta=p.beta, lam=p.lam, w=p.w, eig_mode="topk", K=K, oversample=over,
                         power_iters=q, seed=5, tol=0.0, max_iter=3)
    out = r.prepare(omega=dev(Om, torch.float64)).register()
    U, lam = (host(t) for t in r.export_eig())
    err = np.abs(lam - lo).max() / lo[0]
    say("max |lam - lam_oracle| / lam_1", err, "t_eig", out.t_eig)
    np.testing.assert_allclose(lam, lo, rtol=0, atol=1e-11 * lo[0])
    assert np.all(np.diff(lam) <= 0)
    np.testing.assert_allclose(U.T @ U, np.eye(K), atol=1e-10)
    rows = np.random.default_rng(2).choice(p.M, 40, replace=False)
    Phr = np.exp(-cpd64.sqdist(X[rows], X) / (2 * p.beta ** 2))
    big = lam > 1e-8 * lam[0]
    res = Phr @ U[:, big] - U[rows][:, big] * lam[big]
    assert np.abs(res).max() < 1e-9 * lam[0]


def test_randomized_topk_tiny(lib):
    """40 points, K + p = 12: a single output tile and a single block."""
    import torch
    say("randomized topk tiny")
    p = synth.sphere_pair(M=40, N=45, seed=21)
    X = _f32(p.X)
    K, over, q = 8, 4, 2
    Om = synth.gaussian_matrix(p.M, K + over, seed=3)
    Uo, lo = eig64.eig_topk(X, p.beta, K, Om, power_iters=q)
    r = lib.Registration(dev(X, torch.float32), dev(_f32(p.Y), torch.float32), precision="fp32",
                         beta=p.beta, lam=p.lam, w=p.w, eig_mode="topk", K=K, oversample=over,
                         power_iters=q, seed=5, tol=0.0, max_iter=5)
    r.prepare(omega=dev(Om, torch.float64))
    U, lam = (host(t) for t in r.export_eig())
    np.testing.assert_allclose(lam, lo, rtol=0, atol=1e-11 * lo[0])
    np.testing.assert_allclose(U.T @ U, np.eye(K), atol=1e-10)


def test_full_mode_above_dense_limit(lib):
    """FULL mode at 3000 points (randomized, width grown to round-off) gives
    the registration of the dense eigendecomposition."""
    import torch
    say("full adaptive M=3000")
    p = synth.surface_pair(M=3000, N=3100, seed=4)
    X, Y = _f32(p.X), _f32(p.Y)
    ref = cpd64.register(X, Y, p.beta, p.lam, p.w, "fast",
                         eig=eig64.eig_full(eig64.gram(X, p.beta)), iters=20)
    r = lib.Registration(dev(X, torch.float32), dev(Y, torch.float32), precision="fp32",
                         beta=p.beta, lam=p.lam, w=p.w, eig_mode="full", tol=0.0, max_iter=20)
    out = r.prepare().register()
    say("K", r.K, "t_eig", out.t_eig)
    err = cpd64.rel_rms(host(out.Xt), ref.Xt)
    say("rel_rms", err)
    assert err < 1e-5


def test_full_mode_reports_a_truncated_decomposition(lib):
    """Above 1024 points FULL mode widens its randomized basis up to 2048
    columns.  With a narrow kernel (beta = 0.05 on 3000 unit-sphere points)
    Phi's spectrum decays slowly and even that basis ends far above
    round-off: the call must say so (CPD_NOT_CONVERGED, a message naming the
    trailing Ritz value) and leave a usable top-2016 decomposition
    (orthonormal vectors, eigenvalues descending within Phi's trace)."""
    import torch
    p = synth.sphere_pair(M=3000, seed=21)
    say("truncated FULL, M", p.M, "beta 0.05")
    r = lib.Registration(dev(p.X, torch.float64), dev(p.Y, torch.float64), precision="fp64",
                         beta=0.05, lam=p.lam, w=p.w, eig_mode="full", tol=0.0, max_iter=2)
    with pytest.warns(UserWarning, match="truncated"):
        r.prepare()
    assert r.eig_truncated and "trailing Ritz value" in r.eig_message
    U, lam = (host(t) for t in r.export_eig())
    assert U.shape[1] == r.K == 2016
    assert lam[-1] > 1e-6 * lam[0]
    assert np.all(np.diff(lam) <= 0) and lam.sum() <= p.M
    assert np.abs(U.T @ U - np.eye(U.shape[1])).max() < 1e-10
    r.step()  # still usable
