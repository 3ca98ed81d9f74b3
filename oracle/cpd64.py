"""FP64 reference for one EM iteration of CPD and of Fast CPD.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy / scipy,
float64 throughout, written for a reader checking it against the paper by eye.
Letters follow the paper: X (M x D) is the model set that moves, Y (N x D) the
scene set, Xt = f(X) the transformed model, W the Gaussian-RBF coefficients.

The only structure added beyond the equations is a split of the scene set into
column chunks so that M x N arrays never have to exist whole at large sizes;
every quantity is still the plain sum over all M x N pairs.

Readings of passages where the paper is silent or garbled (each is also listed
with its reason in the design notes):
  * log-domain evaluation of eq. 4-5: mathematically the same p_mn, no 0/0
    when every exp underflows (rows far from all scene points);
  * eq. 5 applied as a row normalisation of the eq. 4 posterior:
    P' = d(P1)^-1 P, so that sum_n p'_mn = 1 and Yt = P'Y;
  * eq. 18 read with P' everywhere: sigma^2 = sum_mn p'_mn |y_n - xt_m|^2/(DM);
  * the original-CPD sigma^2 (eq. 21 comparator) uses N_P = sum(P) in place of
    M (the form eq. 18 takes without the constraint);
  * sigma^2_0 = sum_mn |y_n - xt_m|^2 / (DMN) when no initial value is given;
  * negative round-off eigenvalues of the PSD Gram matrix are clamped to 0;
  * P1 entries are floored at 1e-20 before the inverse in eq. 21.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
from scipy.special import logsumexp

P1_FLOOR = 1e-20


def threads() -> int:
    n = os.environ.get("ORACLE_THREADS")
    return int(n) if n else max(1, min(16, os.cpu_count() or 1))


def _pmap(fn, items):
    items = list(items)
    if len(items) <= 1 or threads() == 1:
        return [fn(i) for i in items]
    with ThreadPoolExecutor(threads()) as ex:
        return list(ex.map(fn, items))


def _chunks(n, size):
    return [(s, min(n, s + size)) for s in range(0, n, size)]


def _auto_chunk(M):
    # keep an M x chunk float64 block around 32 MB
    return int(max(64, min(65536, (4 << 20) // max(M, 1))))


def sqdist(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """|a_i - b_j|^2 by direct differences (no norm expansion)."""
    diff = A[:, None, :] - B[None, :, :]
    return np.einsum("ijk,ijk->ij", diff, diff)


def log_c(sigma2: float, D: int, w: float, M: int, N: int) -> float:
    """Natural log of the outlier constant of eq. 4:
    c = (2 pi sigma^2)^(D/2) * w/(1-w) * M/N.  w = 0 gives c = 0 (-inf)."""
    if w == 0.0:
        return -math.inf
    return (0.5 * D * math.log(2.0 * math.pi * sigma2) + math.log(w)
            - math.log1p(-w) + math.log(M) - math.log(N))


def sigma2_init(Xt: np.ndarray, Y: np.ndarray) -> float:
    """sigma^2_0 = sum_{m,n} |y_n - xt_m|^2 / (D M N) (standard CPD start)."""
    M, D = Xt.shape
    N = Y.shape[0]
    tot = sum(_pmap(lambda se: sqdist(Xt, Y[se[0]:se[1]]).sum(),
                    _chunks(N, _auto_chunk(M))))
    return float(tot) / (D * M * N)


@dataclass
class EStep:
    """Everything one E-step produces (eq. 4 and eq. 5)."""
    logd: np.ndarray    # (N,) log of eq. 4's denominator: log(sum_k e_kn + c)
    o: np.ndarray       # (N,) outlier posterior c/d_n ( = 1 - P^T 1 )
    logr: np.ndarray    # (M,) log of P1_m = sum_n p_mn
    Yt: np.ndarray      # (M,D) P'Y with P' = d(P1)^-1 P   (eq. 5 applied)
    tbar: np.ndarray    # (M,) sum_n p'_mn |y_n - xt_m|^2
    logc: float

    @property
    def P1(self) -> np.ndarray:
        return np.exp(self.logr)

    @property
    def PY(self) -> np.ndarray:
        return self.P1[:, None] * self.Yt

    @property
    def Pt1(self) -> np.ndarray:
        return 1.0 - self.o


def estep(Xt: np.ndarray, Y: np.ndarray, sigma2: float, w: float,
          chunk: int | None = None, rows: np.ndarray | None = None) -> EStep:
    """Eq. 4 posterior with the eq. 5 row constraint, evaluated in log space.

    a_mn   = -|y_n - xt_m|^2 / (2 sigma^2)
    log d_n = logsumexp(a_1n .. a_Mn, log c)                   (eq. 4 denominator)
    log p_mn = a_mn - log d_n                                  (eq. 4)
    log r_m  = logsumexp_n log p_mn,  p'_mn = p_mn / r_m       (eq. 5)
    Yt_m = sum_n p'_mn y_n ;  tbar_m = sum_n p'_mn |y_n - xt_m|^2

    rows: evaluate the row quantities (logr, Yt, tbar) for these model rows
    only; log d_n still sums over every model point.
    """
    M, D = Xt.shape
    N = Y.shape[0]
    lc = log_c(sigma2, D, w, M, N)
    chunk = chunk or _auto_chunk(M)
    cks = _chunks(N, chunk)
    inv2s = 1.0 / (2.0 * sigma2)

    # column pass: log d_n (a column-local reduction over m)
    def col(se):
        s, e = se
        A = -sqdist(Xt, Y[s:e]) * inv2s
        with np.errstate(divide="ignore"):
            ext = np.vstack([A, np.full((1, e - s), lc)])
        return logsumexp(ext, axis=0)
    logd = np.concatenate(_pmap(col, cks))
    if rows is not None:
        Xt = Xt[rows]

    # row pass 1: row maxima of log p_mn
    def rowmax(se):
        s, e = se
        A = -sqdist(Xt, Y[s:e]) * inv2s
        return (A - logd[None, s:e]).max(axis=1)
    mx = np.max(np.stack(_pmap(rowmax, cks)), axis=0)

    # row pass 2: shifted sums
    def rowsum(se):
        s, e = se
        D2 = sqdist(Xt, Y[s:e])
        E = np.exp(-D2 * inv2s - logd[None, s:e] - mx[:, None])
        return E.sum(1), E @ Y[s:e], (E * D2).sum(1)
    parts = _pmap(rowsum, cks)
    S = sum(p[0] for p in parts)
    SY = sum(p[1] for p in parts)
    ST = sum(p[2] for p in parts)
    logr = mx + np.log(S)
    with np.errstate(divide="ignore"):
        o = np.exp(lc - logd) if np.isfinite(lc) else np.zeros(N)
    return EStep(logd=logd, o=o, logr=logr, Yt=SY / S[:, None],
                 tbar=ST / S, logc=lc)


def posterior_dense(Xt, Y, sigma2, w):
    """Small sizes only: the full eq. 4 matrix P (M x N) and the outlier column."""
    M, D = Xt.shape
    N = Y.shape[0]
    lc = log_c(sigma2, D, w, M, N)
    A = -sqdist(Xt, Y) / (2.0 * sigma2)
    with np.errstate(divide="ignore"):
        logd = logsumexp(np.vstack([A, np.full((1, N), lc)]), axis=0)
        o = np.exp(lc - logd) if np.isfinite(lc) else np.zeros(N)
    return np.exp(A - logd[None, :]), o


def fast_mstep(X: np.ndarray, Yt: np.ndarray, U: np.ndarray, lam: np.ndarray,
               lmbda: float, sigma2: float):
    """Eq. 17 (U: all eigenvectors) or eq. 20 (U: the top-K).

    W  = U (Lam + lmbda sigma^2 I)^-1 U^T (Yt - X)
    Xt = X + Phi W, written X + U Lam (Lam + lmbda sigma^2 I)^-1 U^T (Yt - X)
    with Lam clamped at 0.
    """
    lp = np.maximum(lam, 0.0)
    g = 1.0 / (lp + lmbda * sigma2)
    T = U.T @ (Yt - X)
    W = U @ (g[:, None] * T)
    Xt = X + U @ ((lp * g)[:, None] * T)
    return W, Xt


def inverse_mstep(X, Yt, Phi, lmbda, sigma2):
    """Eq. 15 solved directly: (Phi + lmbda sigma^2 I) W = Yt - X."""
    M = X.shape[0]
    W = np.linalg.solve(Phi + lmbda * sigma2 * np.eye(M), Yt - X)
    return W, X + Phi @ W


def cpd_mstep(X, P1, PY, Phi, lmbda, sigma2):
    """Eq. 21 (original CPD): W = (Phi + lmbda sigma^2 d(P1)^-1)^-1
    (d(P1)^-1 PY - X), by Cholesky; Xt = X + Phi W."""
    p1 = np.maximum(P1, P1_FLOOR)
    A = Phi + lmbda * sigma2 * np.diag(1.0 / p1)
    rhs = PY / p1[:, None] - X
    W = sla.cho_solve(sla.cho_factor(A, lower=True), rhs)
    return W, X + Phi @ W


def cpdl_mstep(X, P1, PY, U, lam, lmbda, sigma2):
    """CPD-L: eq. 21 with Phi replaced by its rank-K approximation
    Phi~ = U diag(lam) U^T (eq. 19, lam clamped at 0), solved as written:
    W = (Phi~ + lmbda sigma^2 d(P1)^-1)^-1 (d(P1)^-1 PY - X) by Cholesky,
    Xt = X + Phi~ W.  Phi~ is formed as an M x M matrix, so this is for the
    sizes a dense factorisation allows."""
    p1 = np.maximum(P1, P1_FLOOR)
    Phit = (U * np.maximum(lam, 0.0)) @ U.T
    A = Phit + lmbda * sigma2 * np.diag(1.0 / p1)
    rhs = PY / p1[:, None] - X
    W = sla.cho_solve(sla.cho_factor(A, lower=True), rhs)
    return W, X + Phit @ W


def nearest(A, B):
    """For every row of A the index of its nearest row of B (squared
    Euclidean distance, lowest index on ties)."""
    out = np.empty(A.shape[0], dtype=np.int64)
    for s, e in _chunks(A.shape[0], 2048):
        out[s:e] = np.argmin(sqdist(A[s:e], B), axis=1)
    return out


def mutual_matches(Fixed, Moved):
    """One-to-one correspondences after a registration of `Moved` onto
    `Fixed`: for every fixed point f the nearest moved point m(f), kept only
    when f is also m(f)'s nearest fixed point (mutual nearest neighbours);
    -1 otherwise."""
    fm = nearest(Fixed, Moved)
    mf = nearest(Moved, Fixed)
    return np.where(mf[fm] == np.arange(Fixed.shape[0]), fm, -1)


def matched_mstep(X, Y, match, Phi, lmbda, sigma2):
    """The transformation from given one-to-one correspondences (the second
    half of the two-way scheme for one-sided occlusion, Section IV-A): eq. 21
    with P1_m = 1 and PY_m = y_match(m) for matched model points and P1_m = 0
    (an infinite penalty, so w_m = 0) for the rest.  On the matched set S:
    (Phi_SS + lmbda sigma^2 I) W_S = Y_match(S) - X_S; then Xt = X + Phi_{:,S} W_S
    moves every model point."""
    S = np.flatnonzero(match >= 0)
    W = np.zeros_like(X)
    if S.size:
        A = Phi[np.ix_(S, S)] + lmbda * sigma2 * np.eye(S.size)
        W[S] = sla.cho_solve(sla.cho_factor(A, lower=True), Y[match[S]] - X[S])
    return W, X + Phi @ W


def register_two_way(X, Y, beta, lmbda, w, **kw):
    """Two-way registration for a scene with missing points (Section IV-A):
    register the scene onto the model first, take the mutual-nearest
    one-to-one correspondences, then solve the model's transformation from
    them (matched_mstep, with sigma^2 from the first registration).
    Returns (Xt, W, match, first-stage result)."""
    from . import eig64
    rev = register(Y, X, beta, lmbda, w, "fast", **kw)
    match = mutual_matches(X, rev.Xt)
    Phi = eig64.gram(X, beta)
    W, Xt = matched_mstep(X, Y, match, Phi, lmbda, rev.sigma2)
    return Xt, W, match, rev


def _weighted_sqdist(Xt_old, Y, sigma2, es: EStep, Xt_new, normalised: bool):
    """sum_mn q_mn |y_n - xt_new_m|^2 with q = p' (normalised) or q = p,
    the posterior taken at (Xt_old, sigma2)."""
    M = Xt_old.shape[0]
    N = Y.shape[0]
    inv2s = 1.0 / (2.0 * sigma2)
    shift = es.logr if normalised else np.zeros(M)

    def part(se):
        s, e = se
        logp = -sqdist(Xt_old, Y[s:e]) * inv2s - es.logd[None, s:e]
        return (np.exp(logp - shift[:, None]) * sqdist(Xt_new, Y[s:e])).sum()
    return float(sum(_pmap(part, _chunks(N, _auto_chunk(M)))))


def sigma2_fast(Xt_old, Y, sigma2, es: EStep, Xt_new) -> float:
    """Eq. 18 with P' in place of P: sum_mn p'_mn |y_n - xt_m|^2 / (D M)."""
    M, D = Xt_old.shape
    return _weighted_sqdist(Xt_old, Y, sigma2, es, Xt_new, True) / (D * M)


def sigma2_cpd(Xt_old, Y, sigma2, es: EStep, Xt_new) -> float:
    """Original CPD: sum_mn p_mn |y_n - xt_m|^2 / (D N_P), N_P = sum_mn p_mn."""
    D = Xt_old.shape[1]
    NP = float(np.exp(es.logr).sum())
    return _weighted_sqdist(Xt_old, Y, sigma2, es, Xt_new, False) / (D * NP)


def loglik(Xt, Y, sigma2, w) -> float:
    """Eq. 3: sum_n log[ w/N + (1-w)/M sum_m g(y_n; xt_m, sigma^2 I) ]."""
    M, D = Xt.shape
    N = Y.shape[0]
    lg = -0.5 * D * math.log(2.0 * math.pi * sigma2)

    def part(se):
        s, e = se
        A = -sqdist(Xt, Y[s:e]) / (2.0 * sigma2) + lg + math.log1p(-w) - math.log(M)
        if w > 0:
            A = np.vstack([A, np.full((1, e - s), math.log(w) - math.log(N))])
        return logsumexp(A, axis=0).sum()
    return float(sum(_pmap(part, _chunks(N, _auto_chunk(M)))))


def rmse(Xt, Y_hat) -> float:
    """Eq. 22: sqrt(mean_m |f(x_m) - y_hat_m|^2)."""
    return float(np.sqrt(((Xt - Y_hat) ** 2).sum(1).mean()))


def rel_rms(A, B) -> float:
    """|A - B|_F / |B - mean_rows(B)|_F: the parity measure on point sets."""
    B = np.asarray(B, np.float64)
    den = np.linalg.norm(B - B.mean(0, keepdims=True))
    if den == 0.0:                       # a single point: uncentred norm
        den = np.linalg.norm(B) or 1.0
    return float(np.linalg.norm(np.asarray(A, np.float64) - B) / den)


@dataclass
class RegResult:
    Xt: np.ndarray
    W: np.ndarray
    sigma2: float
    iters: int
    converged: bool
    trace: list          # per iteration: (sigma2, dsigma2)


def register(X, Y, beta, lmbda, w, method="fast", eig=None, Phi=None,
             W0=None, sigma2_0=None, tol=1e-8, max_iter=1000, iters=None,
             floor_rel=1e-10):
    """EM loop (order within an iteration: E-step at (Xt_k, sigma2_k), M-step
    with lmbda*sigma2_k, Xt_{k+1}, then sigma2_{k+1} from P'_k and Xt_{k+1}).

    method: "fast" (eq. 5 + eq. 17/20; eig = (U, lam)), "cpd" (eq. 21) or
    "cpdl" (eq. 21 with the rank-K Phi~ of eq. 19; eig = (U, lam)).
    iters: run exactly this many iterations (no tolerance stop) when given.
    """
    from . import eig64
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    M, D = X.shape
    if method == "cpd" or W0 is not None:
        Phi = eig64.gram(X, beta) if Phi is None else Phi
    if method in ("fast", "cpdl") and eig is None:
        eig = eig64.eig_full(eig64.gram(X, beta) if Phi is None else Phi)
    Xt = X.copy() if W0 is None else X + Phi @ W0
    s2 = sigma2_init(Xt, Y) if not sigma2_0 else float(sigma2_0)
    floor = floor_rel * s2
    W = np.zeros_like(X) if W0 is None else np.asarray(W0, np.float64).copy()
    trace = []
    n_max = iters if iters is not None else max_iter
    converged = False
    k = 0
    for k in range(1, n_max + 1):
        es = estep(Xt, Y, s2, w)
        if method == "fast":
            W, Xn = fast_mstep(X, es.Yt, eig[0], eig[1], lmbda, s2)
            s2n = sigma2_fast(Xt, Y, s2, es, Xn)
        elif method == "cpdl":
            W, Xn = cpdl_mstep(X, es.P1, es.PY, eig[0], eig[1], lmbda, s2)
            s2n = sigma2_cpd(Xt, Y, s2, es, Xn)
        else:
            W, Xn = cpd_mstep(X, es.P1, es.PY, Phi, lmbda, s2)
            s2n = sigma2_cpd(Xt, Y, s2, es, Xn)
        s2n = max(s2n, floor)
        ds = abs(s2n - s2)
        trace.append((s2n, ds))
        Xt, s2 = Xn, s2n
        if iters is None and ds < tol:
            converged = True
            break
    return RegResult(Xt, W, s2, k, converged, trace)
