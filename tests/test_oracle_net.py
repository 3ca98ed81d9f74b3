"""Pins for the FP64 warm-start network: central finite differences of the
loss against the hand-written backward pass, plus the max-pool tie rule and
the packing order."""
import numpy as np
import pytest

from oracle import net64


def _batch(seed=0, M=12, N=14):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(2):
        X = rng.normal(size=(M, 3))
        Y = X[rng.permutation(M)][:min(M, N)]
        Y = np.vstack([Y, rng.normal(size=(max(0, N - M), 3))]) + 0.1
        V = 0.05 * rng.normal(size=(M, 3))
        out.append((X, Y, V))
    return out


def test_finite_differences_match_backward():
    p = net64.init_params(1, out_scale=0.5)
    # biases nonzero so every term is exercised
    rng = np.random.default_rng(2)
    for n in p:
        if n.startswith("b"):
            p[n] = 0.05 * rng.normal(size=p[n].shape)
    batch = _batch()
    L, G = net64.loss_grad(batch, p, beta=1.0)
    h = 1e-6
    for n, idx in [("W1", (2, 5)), ("b1", (7,)), ("W2", (3, 9)), ("W3", (10, 11)),
                   ("W4", (0, 4)), ("b4", (100,)), ("Wa", (5, 6)), ("Wb", (7, 8)),
                   ("Wc", (9, 1)), ("bh", (3,)), ("Wo", (12, 2)), ("bo", (1,))]:
        q = {k: v.copy() for k, v in p.items()}
        q[n][idx] += h
        Lp, _ = net64.loss_grad(batch, q, 1.0)
        q[n][idx] -= 2 * h
        Lm, _ = net64.loss_grad(batch, q, 1.0)
        fd = (Lp - Lm) / (2 * h)
        assert G[n][idx] == pytest.approx(fd, rel=1e-6, abs=1e-9), n


def test_pack_roundtrip_and_count():
    p = net64.init_params(3)
    flat = net64.pack(p)
    assert flat.size == net64.param_count() == 4 * 256 + 256 + 3 * (256 * 256 + 256) + 3 * 256 * 256 + 256 + 256 * 3 + 3
    q = net64.unpack(flat)
    for n in p:
        np.testing.assert_array_equal(p[n], q[n])


def test_maxpool_ties_go_to_the_lowest_index():
    # identical points: every feature ties; the gradient must land on row 0
    p = net64.init_params(4, out_scale=1.0)
    X = np.zeros((5, 3))
    Y = np.ones((4, 3))
    W0, cache = net64.forward(X, Y, p)
    assert np.all(cache["iX"] == 0) and np.all(cache["iY"] == 0)


def test_zero_output_layer_gives_zero_w0():
    p = net64.init_params(5)
    p["Wo"][:] = 0.0
    W0, _ = net64.forward(np.random.default_rng(0).normal(size=(7, 3)),
                          np.random.default_rng(1).normal(size=(9, 3)), p)
    np.testing.assert_array_equal(W0, 0.0)


def test_bf16_rounding_helper():
    a = np.array([1.0, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -3.0e-3, 0.0, 65504.0])
    r = net64.bf16(a)
    np.testing.assert_array_equal(r[[0, 4]], [1.0, 0.0])
    assert r[1] == 1.0                      # tie rounds to even
    assert r[2] == 1.0 + 2 ** -7            # tie rounds to even (up)
    assert abs(r[3] / a[3] - 1) < 2 ** -8
    assert net64.bf16(np.array([1.0 + 2 ** -7]))[0] == 1.0 + 2 ** -7


def test_bf16_mode_is_close_to_float64():
    p = net64.init_params(1, out_scale=0.5)
    batch = _batch()
    L, G = net64.loss_grad(batch, p, 1.0)
    Lb, Gb = net64.loss_grad(batch, p, 1.0, bf16_storage=True)
    assert Lb == pytest.approx(L, rel=3e-2)


def test_bf16_weights_alone_move_the_float64_gradients_by_percents():
    # The bf16 mode's distance from float64 is a property of bf16 storage, not
    # of any kernel: rounding only the four 256 x 256 weight matrices to
    # bfloat16, everything else float64, already moves the gradient by a
    # few percent (8 instances of one model and one scene point).
    p = net64.init_params(7, out_scale=0.5)
    rng = np.random.default_rng(8)
    for n in p:
        if n.startswith("b"):
            p[n] = 0.02 * rng.normal(size=p[n].shape)
    batch = []
    for _ in range(8):
        x = rng.normal(size=(1, 3))
        x /= np.linalg.norm(x)
        batch.append((x, x + 0.3, 0.2 + 0.05 * rng.normal(size=(1, 3))))
    q = dict(p)
    for n in ("W2", "W3", "W4", "Wa"):
        q[n] = net64.bf16(p[n])
    L, G = net64.loss_grad(batch, p, 2.0)
    Lq, Gq = net64.loss_grad(batch, q, 2.0)
    g, gq = net64.pack(G), net64.pack(Gq)
    rel = np.linalg.norm(gq - g) / np.linalg.norm(g)
    assert 5e-3 < rel < 5e-2
    # the deepest encoder block moves most
    relW1 = np.linalg.norm(Gq["W1"] - G["W1"]) / np.linalg.norm(G["W1"])
    assert relW1 > rel
