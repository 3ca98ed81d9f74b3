"""Seeded synthetic point-set workloads for non-rigid registration.

This module only draws inputs.  It holds none of the registration method's
arithmetic (no posterior, no M-step, no sigma^2 update); both the HIP path and
the CPU oracle consume what it returns.  Every generator is deterministic in
its seed (numpy PCG64).

Workloads (D = 3 throughout):

* ``sphere_pair``   -- model points on the unit sphere plus N(0, 0.01^2)
  jitter; the scene is the model pushed through a random Gaussian-RBF
  displacement field, then a fraction of scene rows replaced by uniform
  outliers in [-1.5, 1.5]^3 and the rows shuffled.
* ``surface_pair``  -- the same, on a random smooth closed surface
  r(u) = 1 + sum of 8 real spherical harmonics (degree 1..4) + radial noise.
* ``batch_pairs``   -- many independent surface pairs of uneven sizes.

The displacement field follows the transformation model the paper registers
with (Section III, eq. 9-10): v(p) = sum_j w_j exp(-|p - c_j|^2 / (2 beta^2)),
with centres c_j = the model points and coefficients w_j ~ N(0, s^2).  It is
evaluated here only to *draw* a deformed scene; nothing downstream reuses it.

Every pair keeps the ground-truth correspondence of each model point
(y_hat_m = x_m + v(x_m), before noise and outliers) for the RMSE of
Section IV eq. 22.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

__all__ = ["PointPair", "sphere_pair", "surface_pair", "batch_pairs", "affine_pair",
           "coef_std", "workload", "gaussian_matrix"]


@dataclass
class PointPair:
    X: np.ndarray            # (M, D) model points, float64
    Y: np.ndarray            # (N, D) scene points, float64 (shuffled rows)
    Y_hat: np.ndarray        # (M, D) ground-truth position of each model point
    beta: float
    lam: float
    w: float
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return self.X.shape[0]

    @property
    def N(self) -> int:
        return self.Y.shape[0]


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _rbf_field(P: np.ndarray, C: np.ndarray, Wc: np.ndarray, beta: float,
               chunk: int = 4096) -> np.ndarray:
    """v(p) = sum_j Wc_j exp(-|p - C_j|^2/(2 beta^2)) for every row p of P."""
    out = np.empty((P.shape[0], Wc.shape[1]))
    inv = 1.0 / (2.0 * beta * beta)
    c2 = (C * C).sum(1)
    starts = list(range(0, P.shape[0], chunk))

    def one(s):
        p = P[s:s + chunk]
        d2 = (p * p).sum(1)[:, None] + c2[None, :] - 2.0 * (p @ C.T)
        np.maximum(d2, 0.0, out=d2)
        d2 *= -inv
        np.exp(d2, out=d2)
        out[s:s + chunk] = d2 @ Wc

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(one, starts))
    return out


def coef_std(M: int) -> float:
    """Coefficient scale s(M) = 0.3*sqrt(500/M): keeps the size of the drawn
    displacement field independent of M (0.3 at M = 500)."""
    return 0.3 * np.sqrt(500.0 / M)


def _unit_sphere(rng, n, D=3):
    u = rng.standard_normal((n, D))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def _real_sph_harm(l, m, theta, phi):
    """Real orthonormal spherical harmonic of degree l, order m.
    theta: polar angle, phi: azimuth."""
    from scipy.special import sph_harm_y
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    c = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return np.sqrt(2.0) * (-1) ** m * np.real(c)
    return np.sqrt(2.0) * (-1) ** m * np.imag(c)


class _Surface:
    """r(u) = 1 + sum_i a_i Y_{l_i m_i}(u): 8 harmonics, l in 1..4, |m| <= l,
    a_i ~ N(0, 0.1^2)."""

    def __init__(self, rng, n_terms=8, amp=0.1):
        self.terms = []
        for _ in range(n_terms):
            l = int(rng.integers(1, 5))
            m = int(rng.integers(-l, l + 1))
            self.terms.append((l, m, float(rng.normal(0.0, amp))))

    def sample(self, rng, n, radial_noise=0.02, r_min=0.3):
        u = _unit_sphere(rng, n)
        theta = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
        phi = np.arctan2(u[:, 1], u[:, 0])
        r = np.ones(n)
        for l, m, a in self.terms:
            r += a * _real_sph_harm(l, m, theta, phi)
        r += rng.normal(0.0, radial_noise, n)
        r = np.maximum(r, r_min)
        return u * r[:, None]


def _finish(rng, X, P, centres, Wc, beta, outlier_frac, noise, field_rms=None,
            outlier_box=1.5):
    """Deform P with the field centred at the model points, add noise and
    outliers, shuffle.  With field_rms the coefficients are rescaled so the
    displacement of the model points has that RMS per coordinate.
    Returns (Y, Y_hat)."""
    vX = _rbf_field(X, centres, Wc, beta)
    scale = 1.0
    if field_rms is not None:
        scale = field_rms / np.sqrt(np.mean(vX ** 2))
    vX *= scale
    vP = vX if P is X else scale * _rbf_field(P, centres, Wc, beta)
    Y = P + vP
    Y_hat = X + vX
    if noise > 0:
        Y = Y + rng.normal(0.0, noise, Y.shape)
    n_out = int(round(outlier_frac * Y.shape[0]))
    if n_out > 0:
        idx = rng.choice(Y.shape[0], n_out, replace=False)
        Y[idx] = rng.uniform(-outlier_box, outlier_box, (n_out, Y.shape[1]))
    perm = rng.permutation(Y.shape[0])
    return np.ascontiguousarray(Y[perm]), Y_hat


def sphere_pair(M=500, N=None, seed=0, beta=2.0, lam=3.0, w=0.1,
                coef=0.3, jitter=0.01, outlier_frac=0.10, noise=0.0):
    """Model on the unit sphere (+N(0, jitter^2)); scene = model + RBF field
    with coefficients N(0, coef^2); outlier_frac of scene rows replaced by
    U[-1.5, 1.5]^3; rows shuffled."""
    rng = np.random.default_rng(seed)
    N = M if N is None else N
    X = _unit_sphere(rng, M) + rng.normal(0.0, jitter, (M, 3))
    Wc = rng.normal(0.0, coef, (M, 3))
    if N == M:
        P = X
    else:
        P = _unit_sphere(rng, N) + rng.normal(0.0, jitter, (N, 3))
    Y, Y_hat = _finish(rng, X, P, X, Wc, beta, outlier_frac, noise)
    return PointPair(np.ascontiguousarray(X), Y, Y_hat, beta, lam, w, seed,
                     {"kind": "sphere", "coef": coef, "outliers": outlier_frac,
                      "noise": noise})


def surface_pair(M=10000, N=None, seed=1, beta=2.0, lam=3.0, w=0.1,
                 field_rms=0.2, outlier_frac=0.05, noise=0.0, radial_noise=0.02,
                 outlier_box=1.5):
    """Model on a random spherical-harmonic surface; scene drawn from the same
    surface (the model itself when N == M, fresh samples otherwise), pushed
    through the RBF field centred at the model points.  The field's
    coefficients are N(0, s^2) with s set so that the displacement of the
    model points has RMS `field_rms` per coordinate (20% of the unit radius by
    default): a smooth non-rigid deformation that keeps the deformed scene
    inside the outlier box."""
    rng = np.random.default_rng(seed)
    N = M if N is None else N
    surf = _Surface(rng)
    X = surf.sample(rng, M, radial_noise)
    Wc = rng.normal(0.0, 1.0, (M, 3))
    P = X if N == M else surf.sample(rng, N, radial_noise)
    Y, Y_hat = _finish(rng, X, P, X, Wc, beta, outlier_frac, noise, field_rms, outlier_box)
    return PointPair(np.ascontiguousarray(X), Y, Y_hat, beta, lam, w, seed,
                     {"kind": "surface", "field_rms": field_rms, "outliers": outlier_frac,
                      "noise": noise, "outlier_box": outlier_box, "harmonics": surf.terms})


def affine_pair(M=4000, seed=0, beta=2.0, lam=3.0, w=0.1, a_std=0.1, t_std=0.1):
    """The scaling experiment's kind of input (Section IV-B): the scene is a
    surface point set (a random spherical-harmonic surface stands in for the
    scanned bunny), the model the same points under a random affine map
    x = A y + t, A = I + N(0, a_std^2) entries, t ~ N(0, t_std^2).  No noise
    or outliers.  Y_hat (the true position of each model point) is the scene
    point it came from; the scene rows are shuffled."""
    rng = np.random.default_rng(seed)
    surf = _Surface(rng)
    Y = surf.sample(rng, M, 0.02)
    A = np.eye(3) + rng.normal(0.0, a_std, (3, 3))
    t = rng.normal(0.0, t_std, 3)
    X = Y @ A.T + t
    perm = rng.permutation(M)
    return PointPair(np.ascontiguousarray(X), np.ascontiguousarray(Y[perm]), Y.copy(), beta, lam,
                     w, seed, {"kind": "affine", "A": A, "t": t})


def batch_pairs(B=256, m_range=(500, 8000), seed0=1000, w=0.1,
                beta_range=(1.0, 3.0), lam_range=(1.0, 5.0),
                outlier_frac=0.05):
    """B independent surface pairs; M_i, N_i ~ U{m_range}, beta_i, lam_i
    uniform in their ranges (instance i uses seed seed0 + i)."""
    out = []
    for i in range(B):
        rng = np.random.default_rng(seed0 + i)
        M = int(rng.integers(m_range[0], m_range[1] + 1))
        N = int(rng.integers(m_range[0], m_range[1] + 1))
        beta = float(rng.uniform(*beta_range))
        lam = float(rng.uniform(*lam_range))
        out.append(surface_pair(M, N, seed=seed0 + i, beta=beta, lam=lam, w=w,
                                outlier_frac=outlier_frac))
    return out


def gaussian_matrix(rows: int, cols: int, seed: int) -> np.ndarray:
    """A seeded N(0, 1) rows x cols float64 matrix (numpy PCG64): the test
    matrix of a randomized eigensolver, or random probe vectors."""
    return np.random.default_rng(seed).standard_normal((rows, cols))


def workload(name: str, **kw) -> PointPair:
    """The named registration workloads.

    small500     sphere, M=N=500, beta=2, lam=3, w=0.1, 10% outliers (FP64)
    surface10k   surface, M=N=10000, beta=2, lam=3, w=0.1, 5% outliers
    surface50k   surface, M=N=50000, beta=1.5, lam=2, w=0.2, 20% outliers,
                 N(0, 0.02^2) scene noise
    warm2000     sphere, M=N=2000, beta=2, lam=3, coefficients s(2000)
    """
    if name == "small500":
        a = dict(M=500, seed=0)
        a.update(kw)
        return sphere_pair(**a)
    if name == "surface10k":
        a = dict(M=10000, seed=1)
        a.update(kw)
        return surface_pair(**a)
    if name == "surface50k":
        a = dict(M=50000, seed=2, beta=1.5, lam=2.0, w=0.2, outlier_frac=0.20,
                 noise=0.02)
        a.update(kw)
        return surface_pair(**a)
    if name == "warm2000":
        a = dict(M=2000, seed=10_000_000, coef=coef_std(2000))
        a.update(kw)
        return sphere_pair(**a)
    raise KeyError(name)
