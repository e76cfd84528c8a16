"""Pins of the FP64 warm-start oracle (MLP forward/backward, Adam, feature
and target rows) against things other than itself: central finite
differences, closed forms of degenerate networks, Adam's first step in
closed form, and exact round trips of the row layouts."""
import numpy as np
import pytest

from oracle import mlp
from paper_2604_07644_amd import workloads as W

TINY = (6, 5, 4, 3, 2)


def _tiny(seed=0):
    rng = np.random.default_rng(seed)
    th = rng.standard_normal(mlp.n_params(TINY)) * 0.7
    X = rng.standard_normal((9, 6)); T = rng.standard_normal((9, 2))
    M = (rng.random((9, 2)) < 0.7).astype(float); M[0, 0] = 1
    return th, X, T, M


def test_param_count_matches_layout():
    assert mlp.n_params() == 160 * 512 + 512 + 2 * (512 * 512 + 512) + 512 * 192 + 192
    assert W.ws_init(0).size == mlp.n_params()


def test_gradient_matches_central_differences():
    th, X, T, M = _tiny()
    L, g = mlp.loss_grad(th, X, T, M, TINY)
    assert abs(L - mlp.loss(th, X, T, M, TINY)) < 1e-14
    h = 1e-6
    fd = np.empty_like(th)
    for i in range(th.size):
        e = np.zeros_like(th); e[i] = h
        fd[i] = (mlp.loss(th + e, X, T, M, TINY) - mlp.loss(th - e, X, T, M, TINY)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_all_relus_open_is_affine_composition():
    """Positive inputs, weights and biases keep every ReLU open, so the net is
    the composition of its affine maps."""
    rng = np.random.default_rng(3)
    th = np.abs(rng.standard_normal(mlp.n_params(TINY)))
    X = np.abs(rng.standard_normal((4, 6)))
    Y, _ = mlp.forward(th, X, TINY)
    ref = X
    for Wm, b in mlp.unflatten(th, TINY):
        ref = ref @ Wm + b
    np.testing.assert_allclose(Y, ref, rtol=1e-13)


def test_closed_relu_layer_gives_output_bias():
    """A hidden layer whose pre-activations are all negative outputs zero,
    so Y = b4 and the gradients of everything before it vanish."""
    th, X, T, M = _tiny(1)
    layers = mlp.unflatten(th, TINY)
    Wm, b = layers[2]
    Wm[:] = 0.0; b[:] = -1.0
    Y, _ = mlp.forward(th, X, TINY)
    np.testing.assert_array_equal(Y, np.broadcast_to(layers[3][1], Y.shape))
    _, g = mlp.loss_grad(th, X, T, M, TINY)
    n_before = 6 * 5 + 5 + 5 * 4 + 4 + 4 * 3 + 3
    assert np.all(g[:n_before] == 0.0)


def test_mask_excludes_entries():
    th, X, T, M = _tiny(2)
    Y, _ = mlp.forward(th, X, TINY)
    T2 = np.where(M > 0, T, T + 100.0)
    assert mlp.loss(th, X, T2, M, TINY) == pytest.approx(mlp.loss(th, X, T, M, TINY), rel=1e-15)
    assert mlp.loss(th, X, Y, M, TINY) == 0.0


def test_adam_first_step_closed_form_and_convergence():
    rng = np.random.default_rng(4)
    th = rng.standard_normal(7); g = rng.standard_normal(7)
    t1, m, v = mlp.adam(th, g, np.zeros(7), np.zeros(7), 1, lr=0.01)
    # bias-corrected first moments are g and g^2
    np.testing.assert_allclose(t1, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    # minimising 0.5 |theta - c|^2 converges to c
    c = rng.standard_normal(7)
    th = np.zeros(7); m = np.zeros(7); v = np.zeros(7)
    for t in range(1, 3001):
        th, m, v = mlp.adam(th, th - c, m, v, t, lr=0.01)
    np.testing.assert_allclose(th, c, atol=1e-3)


def _box_small():
    p = W.box_lq(N=6, nx=4, nu=2, xmax=4.0, umax=0.5)
    return p


def test_feature_rows_definition():
    p = _box_small()
    S = W.ws_sketch()
    F = mlp.features(p, S)
    assert F.shape == (p.N + 1, 160)
    np.testing.assert_allclose(F[:, :4], np.broadcast_to(p.x0 / 4.0, (p.N + 1, 4)))
    assert np.all(F[:, 75] == 4.0 / 5.0) and np.all(F[:, 76] == 0.5)
    np.testing.assert_allclose(F[:, 141], np.arange(p.N + 1) / p.N)
    assert np.all(F[:, 4:75] == 0) and np.all(F[:, 145:] == 0)
    assert np.all(F[p.N, 77:141] == 0)
    # the sketch is linear in x0 (with the scaling by x_max held fixed)
    F2 = mlp.features(p, S, x0=2 * p.x0)
    np.testing.assert_allclose(F2[:, 77:141], 2 * F[:, 77:141], rtol=1e-12, atol=1e-15)
    # stage 0's sketch vector written out: (A_0 - I) x0 and B_0^T x0 in their slots
    d = np.zeros(94)
    d[:4] = (p.A[0] - np.eye(4)) @ p.x0 / 4.0
    d[75:77] = p.B[0].T @ p.x0 / 4.0
    np.testing.assert_allclose(F[0, 77:141], S @ d, rtol=1e-12)


def test_targets_and_warm_start_round_trip():
    p = _box_small()
    rng = np.random.default_rng(5)
    z = np.clip(rng.standard_normal(p.m), p.l, p.u)
    lam = rng.standard_normal(p.m)
    T, M = mlp.targets(p, z, lam, rho=3.0)
    assert M.sum() == 2 * p.m + (p.N + 1) * mlp.RHO_WEIGHT
    z0, y0, rho = mlp.warm_start(p, T)
    assert rho == pytest.approx(3.0, rel=1e-14)
    np.testing.assert_allclose(z0, z, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(y0 * rho, lam, rtol=1e-14)
    # predictions outside the box are projected onto it
    T2 = T.copy(); T2[:, :4] = 10.0
    z1, _, _ = mlp.warm_start(p, T2)
    assert np.all(z1 <= p.u) and np.all(z1 >= p.l)
