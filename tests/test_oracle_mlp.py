"""Pins of the oracle's learned-weight functions: the FP64 MLP (18 -> 32 -> 7) and its analytic
gradient, Adam, BF16 rounding, the input features and jump indicator, and the reconstruction
with externally given blend weights (chi, omega_1..6 of Sec. 3.3)."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2508_08965_amd import workloads as W

GAM = 1.4


def rand_net(seed, scale=0.5):
    g = np.random.default_rng(seed)
    return g.normal(scale=scale, size=O.MLP_NPAR)


def rand_batch(seed, n):
    g = np.random.default_rng(seed)
    X = g.uniform(-1, 1, size=(n, 18))
    z = g.normal(size=(n, 7))
    T = np.zeros((n, 7))
    T[:, 0] = 1 / (1 + np.exp(-z[:, 0]))
    e = np.exp(z[:, 1:])
    T[:, 1:] = e / e.sum(axis=1, keepdims=True)
    return X, T


def test_outputs_are_a_probability_split():
    w = rand_net(1)
    X, _ = rand_batch(2, 64)
    Y, H = O.mlp_forward(w, X)
    assert np.all((Y[:, 0] > 0) & (Y[:, 0] < 1))
    assert np.all(Y[:, 1:] > 0)
    np.testing.assert_allclose(Y[:, 1:].sum(axis=1), 1.0, rtol=0, atol=1e-15)
    assert np.all(H >= 0)


def test_zero_network_gives_half_and_equal_weights():
    Y, H = O.mlp_forward(np.zeros(O.MLP_NPAR), rand_batch(3, 5)[0])
    np.testing.assert_array_equal(Y[:, 0], 0.5)
    np.testing.assert_allclose(Y[:, 1:], 1.0 / 6.0, rtol=1e-15)
    assert not H.any()


def test_softmax_shift_invariance_and_chi_independence():
    w = rand_net(4)
    X, _ = rand_batch(5, 32)
    Y0, _ = O.mlp_forward(w, X)
    w2 = w.copy()
    w2[-6:] += 3.7  # the same shift on every omega logit
    Y1, _ = O.mlp_forward(w2, X)
    np.testing.assert_allclose(Y1, Y0, rtol=1e-13, atol=1e-15)
    w3 = w.copy()
    w3[-7] += 1.0  # chi's bias moves chi only
    Y2, _ = O.mlp_forward(w3, X)
    assert np.all(Y2[:, 0] > Y0[:, 0])
    np.testing.assert_array_equal(Y2[:, 1:], Y0[:, 1:])


def test_hidden_layer_brute_force():
    """The hidden activations against a direct evaluation of max(0, W1 x + b1) with numpy's
    matrix product (a library routine, not the oracle's loops)."""
    w = rand_net(6)
    X, _ = rand_batch(7, 40)
    _, H = O.mlp_forward(w, X)
    W1 = w[:32 * 18].reshape(32, 18)
    b1 = w[32 * 18:32 * 18 + 32]
    np.testing.assert_allclose(H, np.maximum(X @ W1.T + b1, 0.0), rtol=1e-13, atol=1e-14)


def test_gradient_matches_central_differences():
    w = rand_net(8)
    X, T = rand_batch(9, 24)
    loss, g = O.mlp_loss_grad(w, X, T)
    assert loss > 0
    h = 1e-6
    fd = np.zeros_like(g)
    for i in range(O.MLP_NPAR):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd[i] = (O.mlp_loss_grad(wp, X, T)[0] - O.mlp_loss_grad(wm, X, T)[0]) / (2 * h)
    err = np.abs(fd - g).max() / np.abs(g).max()
    assert err <= 1e-6, err


def test_loss_is_zero_at_the_targets():
    w = rand_net(10)
    X, _ = rand_batch(11, 16)
    Y, _ = O.mlp_forward(w, X)
    loss, g = O.mlp_loss_grad(w, X, Y)
    assert loss == 0.0
    assert np.abs(g).max() == 0.0


def test_adam_first_step_closed_form_and_convergence():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w0 = np.array([1.0, 2.0, 3.0, 4.0])
    w, m, v = O.adam(w0, np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    # first step: m_hat = g, v_hat = g^2, so w moves by lr g / (|g| + eps)
    np.testing.assert_allclose(w, w0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-12)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)
    # Adam on the quadratic sum (w - c)^2 approaches c
    c = np.array([0.5, -1.5, 2.0])
    w, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        w, m, v = O.adam(w, m, v, 2 * (w - c), t, lr=0.01)
    np.testing.assert_allclose(w, c, atol=1e-3)


def test_bf16_rounding_against_torch_and_ties():
    g = np.random.default_rng(12)
    x = np.concatenate([g.normal(size=1000) * 10.0 ** g.integers(-6, 6, size=1000), [0.0, -0.0, 1.0, -2.5]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.bf16(x), ref)
    # ties go to the even significand
    np.testing.assert_array_equal(O.bf16(np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8])), [1.0, 1 + 2 ** -6])


def _mesh_state(n, prim):
    nodes = W.perturbed_nodes(n, amp=0.05)
    Q, G, L = W.initial_state(nodes, prim, GAM)
    return nodes.numpy(), Q.numpy(), G.numpy(), L.numpy()


def test_features_scale_shift_invariant_and_normalised():
    n = (8, 7, 6)
    nodes, Q, G, L = _mesh_state(n, W.taylor_green(Ma=0.3))
    cells = np.arange(0, Q.shape[1], 5)
    X, jump = O.features(n, nodes, O.params(), Q, L, cells)
    mx = np.abs(X).max(axis=2)
    # rho W of the Taylor-Green field vanishes identically: its features are all zero
    assert np.allclose(mx[:, [0, 1, 2, 4]], 1.0, atol=1e-9) and mx[:, 3].max() < 1e-3
    Q2 = 3.0 * Q + 7.0
    X2, _ = O.features(n, nodes, O.params(), Q2, 3.0 * L, cells)
    np.testing.assert_allclose(X2, X, rtol=0, atol=1e-9)
    assert not jump.any()  # smooth flow at Ma 0.3: no jump


def test_features_uniform_state_and_jump_indicator():
    n = (6, 5, 4)
    nodes, Q, G, L = _mesh_state(n, W.uniform())
    Q[:] = Q[:, :1]  # exactly uniform
    L[:] = 0.0
    X, jump = O.features(n, nodes, O.params(), Q, L, np.arange(Q.shape[1]))
    assert not X.any() and not jump.any()
    nodes, Q, G, L = _mesh_state(n, W.double_sod())
    _, jump = O.features(n, nodes, O.params(), Q, L, np.arange(Q.shape[1]), thresh=0.05)
    assert jump.any() and not jump.all()


def test_recon_with_own_weights_reproduces_geno():
    n = (9, 8, 7)
    nodes, Q, G, L = _mesh_state(n, W.double_sod())
    cells = np.arange(Q.shape[1])
    ref = O.recon(n, nodes, O.params(), Q, G, L, cells)
    gp, wts = O.recon_weights(n, nodes, O.params(), Q, G, L, cells)
    np.testing.assert_array_equal(gp, ref)
    np.testing.assert_allclose(wts[:, :, 1:].sum(axis=2), 1.0, atol=1e-14)
    assert wts[:, :, 0].min() < 0.5  # the discontinuity switches the blend to the linear part
    gp2, wts2 = O.recon_weights(n, nodes, O.params(), Q, G, L, cells, win=wts)
    np.testing.assert_array_equal(gp2, ref)
    np.testing.assert_array_equal(wts2, wts)


def test_recon_with_chi_one_is_the_linear_scheme():
    n = (9, 8, 7)
    nodes, Q, G, L = _mesh_state(n, W.taylor_green(Ma=0.3))
    cells = np.arange(Q.shape[1])
    win = np.zeros((len(cells), 5, 7))
    win[:, :, 0] = 1.0
    win[:, :, 1:] = np.random.default_rng(3).dirichlet(np.ones(6), size=(len(cells), 5))
    gp, _ = O.recon_weights(n, nodes, O.params(), Q, G, L, cells, win=win)
    ref = O.recon(n, nodes, O.params(linear=1), Q, G, L, cells)
    np.testing.assert_array_equal(gp, ref)


def test_recon_with_chi_zero_is_exact_for_linear_fields():
    """chi = 0 keeps only the linear sub-polynomials P_m^1; on a Cartesian mesh every one of
    them is exact for a linear field, so any weights omega reproduce it at the Gauss points."""
    n = (6, 6, 6)
    nodes = W.cartesian_nodes(n)
    a = np.array([0.3, -0.2, 0.1])

    def prim(x, y, z):
        one = torch.ones_like(x)
        rho = 2.0 + a[0] * x + a[1] * y + a[2] * z
        return rho, 0 * one, 0 * one, 0 * one, one

    Q, G, L = W.initial_state(nodes, prim, GAM)
    # interior cells only: the periodic wrap breaks the linear field at the boundary
    idx = [(i, j, k) for k in range(1, 5) for j in range(1, 5) for i in range(1, 5)]
    cells = np.array([i + 6 * (j + 6 * k) for i, j, k in idx])
    win = np.zeros((len(cells), 5, 7))
    win[:, :, 1:] = np.random.default_rng(5).dirichlet(np.ones(6), size=(len(cells), 5))
    gp, _ = O.recon_weights(n, nodes.numpy(), O.params(), Q.numpy(), G.numpy(), L.numpy(), cells, win=win)
    h = 1.0 / 6
    g = 0.5 / math.sqrt(3.0)
    for t, (i, j, k) in enumerate(idx):
        xc = np.array([(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h])
        for m in range(6):
            q, s = m // 2, m % 2
            ta, tb = [ax for ax in range(3) if ax != q]
            for kk in range(4):
                x = xc.copy()
                x[q] += (s - 0.5) * h
                x[ta] += (2 * (kk & 1) - 1) * g * h
                x[tb] += (2 * (kk >> 1) - 1) * g * h
                assert abs(gp[t, 4 * m + kk, 0, 0] - (2.0 + a @ x)) < 1e-13
                np.testing.assert_allclose(gp[t, 4 * m + kk, 0, 1:], a, atol=1e-12)


def test_stage_with_given_weights():
    """A stage with weights given per cell (the learned-weight path of the oracle): GENO's own
    weights reproduce the plain stage bitwise, and chi = 1 everywhere the linear scheme's."""
    n = (9, 8, 7)
    nodes = W.perturbed_nodes(n, amp=0.05)
    Q, G, L = W.initial_state(nodes, W.isotropic_turbulence(16, k0=4.0, Mt=0.6, seed=3), 1.4)
    prm = O.params(viscous=1, mu0=2e-3, Pr=0.72, prandtl_fix=1)
    N = Q.shape[1]
    dt = 0.5 * O.cfl_dt(n, nodes.numpy(), prm, Q.numpy())
    _, wg = O.recon_weights(n, nodes.numpy(), prm, Q.numpy(), G.numpy(), L.numpy(), np.arange(N))
    assert (wg[:, :, 0] < 0.999).any()  # the blend is active somewhere

    def one(stage_fn):
        q, g, l = (np.array(a.numpy()) for a in (Q, G, L))
        stash = np.zeros((90, N))
        assert stage_fn(q, g, l, stash) == 0
        return q, g, l

    plain = one(lambda q, g, l, s: O.stage(n, nodes.numpy(), prm, 1, dt, q, g, l, s))
    given = one(lambda q, g, l, s: O.stage_weights(n, nodes.numpy(), prm, 1, dt, q, g, l, s, wg))
    for a, b in zip(plain, given):
        np.testing.assert_array_equal(a, b)
    ones = wg.copy()
    ones[:, :, 0] = 1.0
    lin = one(lambda q, g, l, s: O.stage(n, nodes.numpy(), O.params(linear=1, viscous=1, mu0=2e-3, Pr=0.72,
                                                                     prandtl_fix=1), 1, dt, q, g, l, s))
    chi1 = one(lambda q, g, l, s: O.stage_weights(n, nodes.numpy(), prm, 1, dt, q, g, l, s, ones))
    for a, b in zip(lin, chi1):
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-13 * np.abs(a).max())
