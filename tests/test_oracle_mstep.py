"""Pins for the oracle's M-steps (Section III, eq. 11-21), sigma^2 (eq. 6,
eq. 18), the eigenpairs (eq. 16, eq. 19) and the EM loops."""
import numpy as np
import pytest
import scipy.optimize as so

import synth
from oracle import cpd64, eig64


def _problem(M=60, N=70, seed=0, beta=1.0, s2=0.3, w=0.2):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (M, 3))
    Y = rng.normal(0, 1, (N, 3))
    es = cpd64.estep(X, Y, s2, w)
    Phi = eig64.gram(X, beta)
    return X, Y, es, Phi


def _Qf(W, X, Y, Pw, Phi, s2, lmbda):
    """Eq. 11 by loops over m: (1/2s2) sum_mn q_mn |y_n - (x_m + phi_m W)|^2
    + lmbda/2 tr(W^T Phi W)."""
    tot = 0.0
    F = X + Phi @ W
    for m in range(X.shape[0]):
        tot += (Pw[m] * ((Y - F[m]) ** 2).sum(1)).sum()
    return tot / (2 * s2) + 0.5 * lmbda * np.trace(W.T @ Phi @ W)


def test_gram_entries():
    X = np.array([[0.0, 0, 0], [np.sqrt(2.0) * 1.5, 0, 0], [0, 0, 3.0]])
    Phi = eig64.gram(X, 1.5)
    assert Phi[0, 1] == pytest.approx(np.exp(-1.0), rel=1e-15)
    assert Phi[0, 2] == pytest.approx(np.exp(-2.0), rel=1e-15)
    np.testing.assert_array_equal(np.diag(Phi), 1.0)
    np.testing.assert_array_equal(Phi, Phi.T)


def test_gram_matmul_matches_dense():
    X = np.random.default_rng(1).normal(size=(300, 3))
    B = np.random.default_rng(2).normal(size=(300, 5))
    np.testing.assert_allclose(eig64.gram_matmul(X, 0.7, B), eig64.gram(X, 0.7) @ B, rtol=1e-12)


def test_full_eig_reconstructs_gram():
    X, _, _, Phi = _problem(200)
    U, lam = eig64.eig_full(Phi)
    M = Phi.shape[0]
    assert np.all(np.diff(lam) <= 0)
    assert np.linalg.norm(U @ np.diag(lam) @ U.T - Phi) / np.linalg.norm(Phi) < 1e-12 * np.sqrt(M)
    assert np.linalg.norm(U.T @ U - np.eye(M)) < 1e-12 * np.sqrt(M)


def test_eq17_equals_the_direct_solve_of_eq15():
    X, Y, es, Phi = _problem()
    U, lam = eig64.eig_full(Phi)
    for s2, lmbda in [(0.3, 2.0), (1e-3, 10.0), (5.0, 0.1)]:
        W, Xt = cpd64.fast_mstep(X, es.Yt, U, lam, lmbda, s2)
        W2 = np.linalg.solve(Phi + lmbda * s2 * np.eye(len(X)), es.Yt - X)
        np.testing.assert_allclose(Phi @ W, Phi @ W2, rtol=1e-9, atol=1e-10 * np.abs(Phi @ W2).max())
        np.testing.assert_allclose(Xt, X + Phi @ W2, rtol=1e-10, atol=1e-10)


def test_eq17_w_is_a_stationary_point_of_eq11():
    X, Y, es, Phi = _problem(M=12, N=15, beta=0.8)
    U, lam = eig64.eig_full(Phi)
    s2, lmbda = 0.3, 2.0
    P = np.exp(-cpd64.sqdist(X, Y) / (2 * s2) - es.logd[None, :])
    Pp = P / P.sum(1, keepdims=True)
    W, _ = cpd64.fast_mstep(X, es.Yt, U, lam, lmbda, s2)
    base = _Qf(W, X, Y, Pp, Phi, s2, lmbda)
    h = 1e-5
    for (i, j) in [(0, 0), (3, 1), (11, 2), (6, 0)]:
        E = np.zeros_like(W)
        E[i, j] = h
        g = (_Qf(W + E, X, Y, Pp, Phi, s2, lmbda) - _Qf(W - E, X, Y, Pp, Phi, s2, lmbda)) / (2 * h)
        assert abs(g) < 1e-6 * max(1.0, base)
    rng = np.random.default_rng(0)
    for _ in range(5):
        assert _Qf(W + 1e-3 * rng.normal(size=W.shape), X, Y, Pp, Phi, s2, lmbda) >= base


def test_eq21_w_is_a_stationary_point_without_the_constraint():
    X, Y, es, Phi = _problem(M=12, N=15, beta=0.8)
    s2, lmbda = 0.3, 2.0
    P = np.exp(-cpd64.sqdist(X, Y) / (2 * s2) - es.logd[None, :])
    W, _ = cpd64.cpd_mstep(X, es.P1, es.PY, Phi, lmbda, s2)
    h = 1e-5
    for (i, j) in [(0, 0), (5, 2), (11, 1)]:
        E = np.zeros_like(W)
        E[i, j] = h
        g = (_Qf(W + E, X, Y, P, Phi, s2, lmbda) - _Qf(W - E, X, Y, P, Phi, s2, lmbda)) / (2 * h)
        assert abs(g) < 1e-6


def test_eq21_with_unit_row_sums_reduces_to_eq15():
    # under the constraint P1 = 1 and PY = Yt, so eq. 21 is eq. 15
    X, Y, es, Phi = _problem()
    s2, lmbda = 0.2, 3.0
    W21, X21 = cpd64.cpd_mstep(X, np.ones(len(X)), es.Yt, Phi, lmbda, s2)
    W15, X15 = cpd64.inverse_mstep(X, es.Yt, Phi, lmbda, s2)
    np.testing.assert_allclose(X21, X15, rtol=1e-10, atol=1e-12)


def test_lambda_limits():
    X, Y, es, Phi = _problem(M=40, N=50, beta=0.5)
    U, lam = eig64.eig_full(Phi)
    _, Xt = cpd64.fast_mstep(X, es.Yt, U, lam, 1e14, 1.0)
    np.testing.assert_allclose(Xt, X, atol=1e-10)
    # Phi is well conditioned at this beta, so lambda -> 0 interpolates Yt
    assert lam.min() > 1e-3
    _, Xt = cpd64.fast_mstep(X, es.Yt, U, lam, 1e-14, 1.0)
    np.testing.assert_allclose(Xt, es.Yt, atol=1e-10)


def test_topk_matches_eigh_and_eckart_young():
    X = synth.workload("small500").X[:400]
    Phi = eig64.gram(X, 2.0)
    U, lam = eig64.eig_full(Phi)
    K = 40
    Om = synth.gaussian_matrix(len(X), K + 10, seed=3)
    Uk, lk = eig64.eig_topk(X, 2.0, K, Om, power_iters=2)
    np.testing.assert_allclose(lk, lam[:K], rtol=1e-10, atol=1e-12 * lam[0])
    err = np.linalg.eigvalsh(Phi - Uk @ np.diag(lk) @ Uk.T)
    assert np.abs(err).max() == pytest.approx(lam[K], rel=1e-6, abs=1e-12 * lam[0])
    np.testing.assert_allclose(Uk.T @ Uk, np.eye(K), atol=1e-12)


def _sigma2_pieces(seed=2):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (25, 3))
    Y = rng.normal(0, 1, (30, 3))
    s2 = 0.4
    es = cpd64.estep(X, Y, s2, 0.15)
    Xn = X + 0.1 * rng.normal(size=X.shape)
    P = np.exp(-cpd64.sqdist(X, Y) / (2 * s2) - es.logd[None, :])
    return X, Y, s2, es, Xn, P


def test_sigma2_fast_brute_trace_and_stable_forms_agree():
    X, Y, s2, es, Xn, P = _sigma2_pieces()
    M, D = X.shape
    Pp = P / P.sum(1, keepdims=True)
    brute = sum(Pp[m, n] * ((Y[n] - Xn[m]) ** 2).sum()
                for m in range(M) for n in range(Y.shape[0])) / (D * M)
    Yt = Pp @ Y
    trace = (np.trace(Y.T @ np.diag(Pp.sum(0)) @ Y) - 2 * np.trace(Yt.T @ Xn)
             + np.trace(Xn.T @ Xn)) / (D * M)       # eq. 18 with P' in place of P
    stable = (es.tbar + 2 * ((es.Yt - X) * (X - Xn)).sum(1) + ((X - Xn) ** 2).sum(1)).sum() / (D * M)
    got = cpd64.sigma2_fast(X, Y, s2, es, Xn)
    for ref in (brute, trace, stable):
        assert got == pytest.approx(ref, rel=1e-12)


def test_sigma2_minimises_the_energy_in_sigma():
    # eq. 6: Q(s2) = S/(2 s2) + (Np D/2) ln s2 with Np = M under the constraint
    X, Y, s2, es, Xn, P = _sigma2_pieces(3)
    M, D = X.shape
    Pp = P / P.sum(1, keepdims=True)
    for Pw, Np, fn in [(Pp, M, cpd64.sigma2_fast), (P, P.sum(), cpd64.sigma2_cpd)]:
        S = sum((Pw[m] * ((Y - Xn[m]) ** 2).sum(1)).sum() for m in range(M))
        res = so.minimize_scalar(lambda v: S / (2 * v) + 0.5 * Np * D * np.log(v),
                                 bounds=(1e-4, 1e2), method="bounded",
                                 options={"xatol": 1e-12})
        assert fn(X, Y, s2, es, Xn) == pytest.approx(res.x, rel=1e-6)


def test_identical_sets_are_a_fixed_point():
    X = synth.workload("small500").X[:200]
    Phi = eig64.gram(X, 2.0)
    U, lam = eig64.eig_full(Phi)
    h = np.sqrt(cpd64.sqdist(X, X)[~np.eye(len(X), dtype=bool)].min())
    r = cpd64.register(X, X, 2.0, 3.0, 0.1, "fast", eig=(U, lam),
                       sigma2_0=1e-4 * h * h, iters=1)
    np.testing.assert_allclose(r.Xt, X, atol=1e-12)
    assert np.abs(Phi @ r.W).max() < 1e-12
    r = cpd64.register(X, X, 2.0, 3.0, 0.1, "fast", eig=(U, lam))
    assert cpd64.rel_rms(r.Xt, X) < 1e-6


def test_translation_is_recovered():
    X = synth.workload("small500").X[:300]
    Y = X + np.array([0.3, -0.2, 0.1])
    Phi = eig64.gram(X, 2.0)
    r = cpd64.register(X, Y, 2.0, 3.0, 0.1, "fast", eig=eig64.eig_full(Phi))
    assert cpd64.rmse(r.Xt, Y) < 1e-3


def test_original_cpd_em_never_increases_its_penalised_nll():
    # EM theorem for the original method: -ln p(Y) + lmbda/2 tr(W^T Phi W)
    p = synth.workload("small500")
    X, Y = p.X[:150], p.Y[:160]
    Phi = eig64.gram(X, p.beta)
    Xt = X.copy()
    s2 = cpd64.sigma2_init(Xt, Y)
    W = np.zeros_like(X)
    prev = -cpd64.loglik(Xt, Y, s2, p.w)
    for _ in range(25):
        es = cpd64.estep(Xt, Y, s2, p.w)
        W, Xn = cpd64.cpd_mstep(X, es.P1, es.PY, Phi, p.lam, s2)
        s2 = cpd64.sigma2_cpd(Xt, Y, s2, es, Xn)
        Xt = Xn
        cur = -cpd64.loglik(Xt, Y, s2, p.w) + 0.5 * p.lam * np.trace(W.T @ Phi @ W)
        assert cur <= prev + 1e-12 * abs(prev)
        prev = cur


def test_rmse_definition():
    A = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    B = np.array([[0.0, 0, 3.0], [1.0, 4.0, 0]])
    assert cpd64.rmse(A, B) == pytest.approx(np.sqrt((9 + 16) / 2))


def test_rel_rms_by_hand():
    # B's rows have mean (1, 0, 0); centred, |B - mean|_F^2 = 1 + 1 = 2.
    # A differs from B by 1 in one entry: rel_rms = 1 / sqrt(2)
    B = np.array([[0.0, 0, 0], [2.0, 0, 0]])
    A = np.array([[0.0, 1, 0], [2.0, 0, 0]])
    assert cpd64.rel_rms(A, B) == pytest.approx(1.0 / np.sqrt(2.0), rel=1e-15)
    # a common translation of both sets changes nothing (centred denominator)
    t = np.array([100.0, -50.0, 7.0])
    assert cpd64.rel_rms(A + t, B + t) == pytest.approx(1.0 / np.sqrt(2.0), rel=1e-12)
    # errors of 3 and 4 over a set with centred norm 10 (rows -5, +5, 0 in x)
    B = np.array([[-5.0, 0, 0], [5.0, 0, 0], [0.0, 0, 0]])
    A = B + np.array([[0.0, 3, 0], [0.0, 0, 4], [0.0, 0, 0]])
    assert cpd64.rel_rms(A, B) == pytest.approx(5.0 / np.sqrt(50.0), rel=1e-15)
    # it is not symmetric: the denominator is the second argument's spread
    assert cpd64.rel_rms(B, A) != pytest.approx(cpd64.rel_rms(A, B))
    # one point: the uncentred norm
    assert cpd64.rel_rms(np.array([[3.0, 4, 0]]), np.array([[0.0, 0, 5.0]])) == \
        pytest.approx(np.sqrt(9 + 16 + 25) / 5.0)
    assert cpd64.rel_rms(B, B) == 0.0


def _low_rank(Phi, K):
    lam, U = np.linalg.eigh(Phi)
    o = np.argsort(lam)[::-1][:K]
    return U[:, o], lam[o]


def test_cpdl_equals_the_matrix_inversion_lemma_form():
    # CPD-L: eq. 21 with Phi~ = U L U^T (eq. 19).  The oracle factorises the
    # M x M matrix; the same W follows from the Sherman-Morrison-Woodbury
    # identity through a K x K system, an independent route:
    #   A = lmbda s2 d(P1)^-1,  t = A^-1 (d(P1)^-1 PY - X),
    #   (A + U L U^T)^-1 = A^-1 - A^-1 U (L^-1 + U^T A^-1 U)^-1 U^T A^-1
    X, Y, es, Phi = _problem(M=50, N=60, beta=1.2)
    s2, lmbda = 0.25, 2.0
    for K in (5, 17, 40):
        U, lam = _low_rank(Phi, K)
        ainv = es.P1 / (lmbda * s2)
        t = ainv[:, None] * (es.PY / es.P1[:, None] - X)
        S = np.diag(1.0 / lam) + U.T @ (ainv[:, None] * U)
        z = np.linalg.solve(S, U.T @ t)
        Ww = t - ainv[:, None] * (U @ z)
        W, Xt = cpd64.cpdl_mstep(X, es.P1, es.PY, U, lam, lmbda, s2)
        np.testing.assert_allclose(W, Ww, rtol=1e-8, atol=1e-10 * np.abs(Ww).max())
        # and Phi~ W collapses to U z (L (U^T t - (S - L^-1) z) = z)
        np.testing.assert_allclose(Xt, X + U @ z, rtol=1e-10, atol=1e-12)


def test_cpdl_drops_pairs_with_negative_eigenvalues():
    # lam <= 0 carries no part of Phi~ (clamped at 0): adding such a pair
    # leaves the result unchanged
    X, Y, es, Phi = _problem(M=30, N=35, beta=1.0)
    U, lam = _low_rank(Phi, 8)
    W, Xt = cpd64.cpdl_mstep(X, es.P1, es.PY, U[:, :7], lam[:7], 2.0, 0.3)
    lam2 = lam.copy()
    lam2[7] = -0.5
    W2, Xt2 = cpd64.cpdl_mstep(X, es.P1, es.PY, U, lam2, 2.0, 0.3)
    np.testing.assert_allclose(Xt2, Xt, rtol=1e-12, atol=1e-13)


def test_cpdl_at_full_rank_is_the_original_mstep():
    X, Y, es, Phi = _problem(M=40, N=45, beta=0.6)   # Phi well conditioned
    s2, lmbda = 0.3, 1.5
    U, lam = _low_rank(Phi, 40)
    assert lam.min() > 1e-8
    W, Xt = cpd64.cpdl_mstep(X, es.P1, es.PY, U, lam, lmbda, s2)
    W21, X21 = cpd64.cpd_mstep(X, es.P1, es.PY, Phi, lmbda, s2)
    np.testing.assert_allclose(Xt, X21, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(W, W21, rtol=1e-6, atol=1e-8 * np.abs(W21).max())


def test_cpdl_w_is_a_stationary_point_of_the_rank_k_objective():
    # eq. 11's objective with the unnormalised posterior and Phi~ in place of
    # Phi: its gradient in W vanishes at CPD-L's W (finite differences)
    X, Y, es, Phi = _problem(M=12, N=15, beta=0.8)
    s2, lmbda = 0.3, 2.0
    U, lam = _low_rank(Phi, 6)
    Pt = (U * lam) @ U.T
    P = np.exp(-cpd64.sqdist(X, Y) / (2 * s2) - es.logd[None, :])
    W, _ = cpd64.cpdl_mstep(X, es.P1, es.PY, U, lam, lmbda, s2)
    h = 1e-5
    for (i, j) in [(0, 0), (5, 2), (11, 1)]:
        E = np.zeros_like(W)
        E[i, j] = h
        g = (_Qf(W + E, X, Y, P, Pt, s2, lmbda) - _Qf(W - E, X, Y, P, Pt, s2, lmbda)) / (2 * h)
        assert abs(g) < 1e-6


def test_cpdl_registration_runs_and_lowers_sigma2():
    p = synth.sphere_pair(M=120, N=130, seed=5, coef=0.05)
    U, lam = _low_rank(eig64.gram(p.X, p.beta), 30)
    r = cpd64.register(p.X, p.Y, p.beta, p.lam, p.w, "cpdl", eig=(U, lam), iters=30)
    s = [t[0] for t in r.trace]
    assert np.all(np.isfinite(r.Xt)) and s[-1] < 0.1 * s[0]


def test_nearest_and_mutual_matches_by_loops():
    rng = np.random.default_rng(9)
    F = rng.normal(size=(9, 3))
    Mv = rng.normal(size=(7, 3))
    Mv[3] = Mv[1]                     # a tie: the lower index wins
    nn = cpd64.nearest(F, Mv)
    for i in range(9):
        d = [((F[i] - Mv[j]) ** 2).sum() for j in range(7)]
        assert nn[i] == int(np.argmin(d))
    mt = cpd64.mutual_matches(F, Mv)
    for i in range(9):
        j = nn[i]
        back = int(np.argmin([((Mv[j] - F[k]) ** 2).sum() for k in range(9)]))
        assert mt[i] == (j if back == i else -1)
    assert 3 not in set(mt)


def test_matched_mstep_with_identity_matches_is_eq15():
    # every model point matched one-to-one: eq. 21 with P1 = 1 and PY = the
    # matched scene points, i.e. eq. 15 with Yt = Y[match]
    X, Y, es, Phi = _problem(M=30, N=30)
    s2, lmbda = 0.2, 3.0
    match = np.random.default_rng(2).permutation(30)
    W, Xt = cpd64.matched_mstep(X, Y, match, Phi, lmbda, s2)
    W15, X15 = cpd64.inverse_mstep(X, Y[match], Phi, lmbda, s2)
    np.testing.assert_allclose(Xt, X15, rtol=1e-10, atol=1e-12)


def test_matched_mstep_is_the_limit_of_eq21_with_vanishing_weights():
    # unmatched rows: P1 -> 0 in eq. 21 drives their W to 0; the matched-set
    # solve is that limit (P1 = 1e-12 on unmatched rows, PY = P1 Y[match])
    X, Y, es, Phi = _problem(M=40, N=35, beta=0.9)
    s2, lmbda = 0.3, 2.0
    rng = np.random.default_rng(3)
    match = np.where(rng.random(40) < 0.6, rng.integers(0, 35, 40), -1)
    W, Xt = cpd64.matched_mstep(X, Y, match, Phi, lmbda, s2)
    P1 = np.where(match >= 0, 1.0, 1e-12)
    PY = P1[:, None] * np.where(match[:, None] >= 0, Y[np.maximum(match, 0)], 0.0)
    W21, X21 = cpd64.cpd_mstep(X, P1, PY, Phi, lmbda, s2)
    np.testing.assert_allclose(Xt, X21, rtol=1e-7, atol=1e-9)


def test_two_way_recovers_a_deformation_with_missing_scene_points():
    # the scene lacks a third of the model's points (one-sided occlusion):
    # the two-way result is closer to the truth than the direct registration
    p = synth.sphere_pair(M=300, N=300, seed=4, coef=0.03, outlier_frac=0.0)
    keep = p.Y[:, 2] < 0.35                      # cut the scene's top cap
    Y = p.Y[keep]
    direct = cpd64.register(p.X, Y, p.beta, p.lam, 0.1, "fast", iters=60)
    Xt, W, match, rev = cpd64.register_two_way(p.X, Y, p.beta, p.lam, 0.1, iters=60)
    e_direct = cpd64.rmse(direct.Xt, p.Y_hat)
    e_two = cpd64.rmse(Xt, p.Y_hat)
    assert (match >= 0).sum() > 0.3 * Y.shape[0]
    assert e_two < e_direct
