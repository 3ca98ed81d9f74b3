"""FP64 reference of the learned warm-start network and its gradients.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, float64.

The network maps a model set X (M x 3) and a scene set Y (N x 3) to initial
Gaussian-RBF coefficients W0 (M x 3) for the transformation f(X) = X + Phi W
(Section III, eq. 9-11); registration then starts from Xt_0 = X + Phi W0.

  encoder  shared per-point MLP on e = [p, flag] (flag 0 model, 1 scene):
           h1 = relu(e W1 + b1), h2 = relu(h1 W2 + b2), h3 = relu(h2 W3 + b3),
           f = relu(h3 W4 + b4)                         (4 -> 256 -> 256 -> 256 -> 256)
  pool     g_X = max over model points of f, g_Y = max over scene points
           (ties: the lowest index receives the gradient)
  head     z = relu(f(x_m) Wa + g_X Wb + g_Y Wc + bh),  W0_m = z Wo + bo
  loss     L = mean over the batch of |Phi W0 - V*|_F^2 / M, V* the true
           displacement of the model points.  W itself is not identifiable
           (Phi is numerically low rank), the displacement Phi W is.

Parameters are a dict of float64 arrays with the shapes above (W as
[fan_in, fan_out]); `pack`/`unpack` use the flat order PARAM_ORDER, which the
GPU library uses for its FP32 master copy.
"""
from __future__ import annotations

import numpy as np

from .eig64 import gram

H = 256
PARAM_SHAPES = [
    ("W1", (4, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
    ("W4", (H, H)), ("b4", (H,)), ("Wa", (H, H)), ("Wb", (H, H)), ("Wc", (H, H)), ("bh", (H,)),
    ("Wo", (H, 3)), ("bo", (3,)),
]
PARAM_ORDER = [n for n, _ in PARAM_SHAPES]


def param_count() -> int:
    return int(sum(np.prod(s) for _, s in PARAM_SHAPES))


def pack(params) -> np.ndarray:
    return np.concatenate([np.asarray(params[n], np.float64).ravel() for n in PARAM_ORDER])


def unpack(flat) -> dict:
    out, o = {}, 0
    for n, s in PARAM_SHAPES:
        k = int(np.prod(s))
        out[n] = np.asarray(flat[o:o + k], np.float64).reshape(s)
        o += k
    return out


def relu(a):
    return np.maximum(a, 0.0)


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(a):
    return a


def encode(P, flag, p, r=_ident):
    e = np.concatenate([P, np.full((P.shape[0], 1), float(flag))], axis=1)
    h1 = r(relu(e @ p["W1"] + p["b1"]))
    h2 = r(relu(h1 @ r(p["W2"]) + p["b2"]))
    h3 = r(relu(h2 @ r(p["W3"]) + p["b3"]))
    f = r(relu(h3 @ r(p["W4"]) + p["b4"]))
    return e, (h1, h2, h3, f)


def forward(X, Y, p, r=_ident):
    """W0 (M x 3) and the cache the backward pass needs.  r rounds stored
    activations and the 256 x 256 weights (bf16 for the bf16 mode)."""
    eX, aX = encode(X, 0, p, r)
    eY, aY = encode(Y, 1, p, r)
    fX, fY = aX[3], aY[3]
    iX, iY = fX.argmax(0), fY.argmax(0)        # argmax returns the lowest index
    gX, gY = fX[iX, np.arange(H)], fY[iY, np.arange(H)]
    u = gX @ p["Wb"] + gY @ p["Wc"] + p["bh"]
    z = r(relu(fX @ r(p["Wa"]) + u))
    W0 = z @ p["Wo"] + p["bo"]
    cache = dict(eX=eX, aX=aX, eY=eY, aY=aY, iX=iX, iY=iY, gX=gX, gY=gY, z=z)
    return W0, cache


def loss_and_dW(X, W0, V, beta):
    """L = |Phi W0 - V|^2 / M and dL/dW0 = 2 Phi (Phi W0 - V) / M."""
    Phi = gram(X, beta)
    R = Phi @ W0 - V
    M = X.shape[0]
    return float((R * R).sum() / M), 2.0 * (Phi @ R) / M


def _encoder_back(e, acts, df, p, g, r=_ident):
    h1, h2, h3, f = acts
    d = r(df * (f > 0))
    g["W4"] += h3.T @ d
    g["b4"] += d.sum(0)
    d = r((d @ r(p["W4"]).T) * (h3 > 0))
    g["W3"] += h2.T @ d
    g["b3"] += d.sum(0)
    d = r((d @ r(p["W3"]).T) * (h2 > 0))
    g["W2"] += h1.T @ d
    g["b2"] += d.sum(0)
    d = r((d @ r(p["W2"]).T) * (h1 > 0))
    g["W1"] += e.T @ d
    g["b1"] += d.sum(0)


def backward(dW0, cache, p, r=_ident):
    """Gradients of sum(dW0 * W0) with respect to every parameter."""
    g = {n: np.zeros(s) for n, s in PARAM_SHAPES}
    z = cache["z"]
    g["Wo"] += z.T @ dW0
    g["bo"] += dW0.sum(0)
    dz = r((dW0 @ p["Wo"].T) * (z > 0))
    fX = cache["aX"][3]
    g["Wa"] += fX.T @ dz
    du = dz.sum(0)
    g["Wb"] += np.outer(cache["gX"], du)
    g["Wc"] += np.outer(cache["gY"], du)
    g["bh"] += du
    dfX = dz @ r(p["Wa"]).T
    dfY = np.zeros_like(cache["aY"][3])
    dgX, dgY = p["Wb"] @ du, p["Wc"] @ du
    dfX[cache["iX"], np.arange(H)] += dgX
    dfY[cache["iY"], np.arange(H)] += dgY
    _encoder_back(cache["eX"], cache["aX"], dfX, p, g, r)
    _encoder_back(cache["eY"], cache["aY"], dfY, p, g, r)
    return g


def loss_grad(batch, p, beta, bf16_storage=False):
    """Mean loss over a batch of (X, Y, V) and its parameter gradients.

    bf16_storage=True evaluates the bf16 precision mode's definition: the
    256 x 256 weights, every stored activation and every backward gradient
    between layers rounded to bfloat16, all sums and the loss in float64."""
    r = bf16 if bf16_storage else _ident
    tot = 0.0
    G = {n: np.zeros(s) for n, s in PARAM_SHAPES}
    for X, Y, V in batch:
        W0, cache = forward(X, Y, p, r)
        L, dW = loss_and_dW(X, W0, V, beta)
        tot += L
        g = backward(dW, cache, p, r)
        for n in G:
            G[n] += g[n]
    B = len(batch)
    return tot / B, {n: G[n] / B for n in G}


def init_params(seed=0, out_scale=1e-3):
    """He-normal weights, zero biases, a small output layer (W0 ~ 0 at start)."""
    rng = np.random.default_rng(seed)
    p = {}
    for n, s in PARAM_SHAPES:
        if n.startswith("b"):
            p[n] = np.zeros(s)
        else:
            std = np.sqrt(2.0 / s[0]) * (out_scale if n == "Wo" else 1.0)
            p[n] = rng.normal(0.0, std, s)
    return p
