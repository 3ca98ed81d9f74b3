"""Pins for the oracle's E-step (Section II, eq. 1-5) and log-likelihood (eq. 3).

Each test checks the oracle against something other than its own formula:
Bayes' rule on the mixture of eq. 2, library densities, invariants of the
normalisations, limits with a known answer, and brute force on tiny inputs.
"""
import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal

from oracle import cpd64


def _rand(M, N, D=3, seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, (M, D)), rng.normal(0, scale, (N, D))


def _mixture_posterior(X, Y, s2, w):
    """Posterior of each component of the eq. 2 mixture by Bayes' rule, with
    densities from scipy: p(m | y_n) = (1-w)/M g(y_n; x_m, s2 I) / p(y_n),
    outlier: (w/N) / p(y_n)."""
    M, D = X.shape
    N = Y.shape[0]
    G = np.array([[multivariate_normal.pdf(Y[n], mean=X[m], cov=s2 * np.eye(D))
                   for n in range(N)] for m in range(M)])
    comp = (1 - w) / M * G
    py = comp.sum(0) + w / N
    return comp / py, (w / N) / py, py


@pytest.mark.parametrize("w", [0.0, 0.1, 0.7])
@pytest.mark.parametrize("D", [1, 2, 3])
def test_posterior_is_bayes_rule_of_the_mixture(w, D):
    X, Y = _rand(6, 7, D, seed=D)
    s2 = 0.8
    P_ref, o_ref, _ = _mixture_posterior(X, Y, s2, w)
    es = cpd64.estep(X, Y, s2, w)
    P = np.exp(-cpd64.sqdist(X, Y) / (2 * s2) - es.logd[None, :])
    np.testing.assert_allclose(P, P_ref, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(es.o, o_ref, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(es.P1, P_ref.sum(1), rtol=1e-12)
    np.testing.assert_allclose(es.Pt1, P_ref.sum(0), rtol=1e-12)
    Pp = P_ref / P_ref.sum(1, keepdims=True)
    np.testing.assert_allclose(es.Yt, Pp @ Y, rtol=1e-11, atol=1e-13)
    D2 = np.array([[sum((Y[n][k] - X[m][k]) ** 2 for k in range(D))
                    for n in range(Y.shape[0])] for m in range(X.shape[0])])
    np.testing.assert_allclose(es.tbar, (Pp * D2).sum(1), rtol=1e-11)


def test_dense_posterior_matches_estep():
    X, Y = _rand(9, 11, seed=3)
    P, o = cpd64.posterior_dense(X, Y, 0.5, 0.2)
    es = cpd64.estep(X, Y, 0.5, 0.2)
    np.testing.assert_allclose(P.sum(1), es.P1, rtol=1e-13)
    np.testing.assert_allclose(o, es.o, rtol=1e-13)


def test_columns_with_outlier_mass_sum_to_one():
    # eq. 4: sum_m p_mn + c/d_n = 1 for every scene point n
    X, Y = _rand(120, 150, seed=4)
    es = cpd64.estep(X, Y, 0.3, 0.25)
    P = np.exp(-cpd64.sqdist(X, Y) / 0.6 - es.logd[None, :])
    np.testing.assert_allclose(P.sum(0) + es.o, 1.0, atol=1e-14)


def test_rows_sum_to_one_after_constraint():
    # eq. 5: sum_n p'_mn = 1 for every model point m
    X, Y = _rand(120, 150, seed=5)
    es = cpd64.estep(X, Y, 0.3, 0.25)
    P = np.exp(-cpd64.sqdist(X, Y) / 0.6 - es.logd[None, :])
    Pp = P / np.exp(es.logr)[:, None]
    np.testing.assert_allclose(Pp.sum(1), 1.0, atol=1e-14)


def test_chunking_does_not_change_the_result():
    X, Y = _rand(200, 333, seed=6)
    a = cpd64.estep(X, Y, 0.2, 0.1)
    b = cpd64.estep(X, Y, 0.2, 0.1, chunk=37)
    for f in ("logd", "logr", "Yt", "tbar", "o"):
        np.testing.assert_allclose(getattr(a, f), getattr(b, f), rtol=1e-13, atol=1e-15)


def test_hand_computed_1d_case():
    # D=1, one model point at 0, scene points at -1 and 2, sigma^2 = 1/2,
    # w = 1/2: c = (2 pi 1/2)^(1/2) * 1 * (1/2) = sqrt(pi)/2.
    # e_1 = exp(-1), e_2 = exp(-4); p_n = e_n / (e_n + c) (one model point).
    c = math.sqrt(math.pi) / 2
    p1 = math.exp(-1) / (math.exp(-1) + c)
    p2 = math.exp(-4) / (math.exp(-4) + c)
    es = cpd64.estep(np.array([[0.0]]), np.array([[-1.0], [2.0]]), 0.5, 0.5)
    assert es.P1[0] == pytest.approx(p1 + p2, rel=1e-14)
    assert es.Yt[0, 0] == pytest.approx((-p1 + 2 * p2) / (p1 + p2), rel=1e-14)
    assert es.o == pytest.approx([c / (math.exp(-1) + c), c / (math.exp(-4) + c)], rel=1e-14)
    assert es.logc == pytest.approx(math.log(c), rel=1e-15)


def test_single_pair_maps_onto_the_scene():
    es = cpd64.estep(np.array([[0.3, -1.0, 2.0]]), np.array([[4.0, 5.0, -6.0]]), 0.01, 0.3)
    np.testing.assert_allclose(es.Yt, [[4.0, 5.0, -6.0]])


def test_huge_sigma_gives_the_scene_mean_without_outliers():
    X, Y = _rand(30, 40, seed=7)
    es = cpd64.estep(X, Y, 1e12, 0.0)
    np.testing.assert_allclose(es.Yt, np.broadcast_to(Y.mean(0), es.Yt.shape), rtol=1e-9, atol=1e-9)


def test_w_zero_is_a_column_softmax():
    X, Y = _rand(10, 12, seed=8)
    s2 = 0.4
    es = cpd64.estep(X, Y, s2, 0.0)
    A = -cpd64.sqdist(X, Y) / (2 * s2)
    S = np.exp(A) / np.exp(A).sum(0, keepdims=True)
    np.testing.assert_allclose(es.P1, S.sum(1), rtol=1e-12)
    assert np.all(es.o == 0)


def test_far_model_point_gets_its_nearest_scene_points():
    # every exp underflows for the far row in plain arithmetic; the
    # constrained posterior still concentrates on the nearest scene point
    X = np.array([[0.0, 0, 0], [1e3, 0, 0]])
    Y = np.array([[0.1, 0, 0], [-0.1, 0, 0], [2.0, 0, 0]])
    es = cpd64.estep(X, Y, 1e-2, 0.1)
    assert np.all(np.isfinite(es.Yt))
    np.testing.assert_allclose(es.Yt[1], [2.0, 0, 0], atol=1e-12)


def test_loglik_matches_library_densities():
    X, Y = _rand(8, 9, seed=9)
    s2, w = 0.7, 0.2
    _, _, py = _mixture_posterior(X, Y, s2, w)
    assert cpd64.loglik(X, Y, s2, w) == pytest.approx(np.log(py).sum(), rel=1e-12)


def test_sigma2_init_is_the_mean_square_distance():
    X, Y = _rand(13, 17, seed=10)
    brute = sum(((Y[n] - X[m]) ** 2).sum() for m in range(13) for n in range(17))
    assert cpd64.sigma2_init(X, Y) == pytest.approx(brute / (3 * 13 * 17), rel=1e-13)


def test_row_subset_matches_full_evaluation():
    """estep(rows=...) gives the sampled rows of the full evaluation (log d_n
    still over every model point)."""
    rng = np.random.default_rng(21)
    Y = rng.normal(size=(90, 3))
    Xt = Y[rng.choice(90, 70)] + 0.1 * rng.normal(size=(70, 3))
    full = cpd64.estep(Xt, Y, 0.05, 0.2)
    rows = np.array([3, 17, 40, 69])
    sub = cpd64.estep(Xt, Y, 0.05, 0.2, rows=rows)
    np.testing.assert_allclose(sub.logd, full.logd, rtol=0, atol=1e-13)
    np.testing.assert_allclose(sub.logr, full.logr[rows], rtol=0, atol=1e-13)
    np.testing.assert_allclose(sub.Yt, full.Yt[rows], rtol=1e-13)
    np.testing.assert_allclose(sub.tbar, full.tbar[rows], rtol=1e-12)
