"""FP64 reference for the Gram matrix and its eigenpairs.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  gram(X, beta)            Phi_ij = exp(-|x_i - x_j|^2 / (2 beta^2))   (eq. 11)
  gram_matmul(X, beta, B)  Phi @ B with rows of Phi formed on the fly
  eig_full(Phi)            Phi = U Lam U^T, all M pairs, descending     (eq. 16)
  eig_topk(...)            the K largest pairs (eq. 19) by a randomized
                           range finder with subspace iteration and a
                           Rayleigh-Ritz step (Halko, Martinsson & Tropp,
                           SIAM Review 53(2), 2011).  The Gaussian test matrix
                           Omega is an input (synth.gaussian_matrix draws it),
                           so the same draw can feed the GPU solver.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .cpd64 import _auto_chunk, _chunks, _pmap, sqdist


def gram(X: np.ndarray, beta: float) -> np.ndarray:
    return np.exp(-sqdist(X, X) / (2.0 * beta * beta))


def gram_matmul(X: np.ndarray, beta: float, B: np.ndarray) -> np.ndarray:
    """Phi @ B without storing Phi (row blocks of Phi built on the fly)."""
    M = X.shape[0]
    out = np.empty((M, B.shape[1]))
    inv = 1.0 / (2.0 * beta * beta)

    def part(se):
        s, e = se
        out[s:e] = np.exp(-sqdist(X[s:e], X) * inv) @ B
    _pmap(part, _chunks(M, _auto_chunk(M)))
    return out


def eig_full(Phi: np.ndarray):
    """All eigenpairs of the symmetric Gram matrix, eigenvalues descending.
    Returns (U, lam); lam may hold tiny negative round-off values (callers
    clamp at 0)."""
    lam, U = sla.eigh(Phi)
    order = np.argsort(lam)[::-1]
    return np.ascontiguousarray(U[:, order]), lam[order]


def _orth(Z):
    Q, _ = np.linalg.qr(Z)
    return Q


def eig_topk(X: np.ndarray, beta: float, K: int, Omega: np.ndarray,
             power_iters: int = 2):
    """Top-K eigenpairs of Phi(X, beta).

    Q   = orth(Phi Omega)                 range finder, Omega is M x (K + p)
    Q   = orth(Phi Q)      (power_iters times: subspace iteration)
    B   = Q^T Phi Q,  B = S Theta S^T     Rayleigh-Ritz
    U~  = Q S[:, :K],  Lam~ = Theta[:K]   (descending)
    """
    Q = _orth(gram_matmul(X, beta, Omega))
    for _ in range(power_iters):
        Q = _orth(gram_matmul(X, beta, Q))
    B = Q.T @ gram_matmul(X, beta, Q)
    B = 0.5 * (B + B.T)
    theta, S = sla.eigh(B)
    order = np.argsort(theta)[::-1][:K]
    return np.ascontiguousarray(Q @ S[:, order]), theta[order]

