"""Pins of the oracle's compact reconstruction (Sec. 3.2-3.3, Sec. 4).

  * the constrained least-squares matrix R against an independent 40-digit null-space
    solution of eq. (compact-big-ref) (h1'=2, h2'=1, h3'=3; exact face-neighbour rows);
  * polynomial exactness: data of any quartic on Cartesian and affine meshes reproduce its
    point values and gradients at the 24 face Gauss points (values computed here from the
    polynomial itself, by the test);
  * the smoothness Gram matrices against exact symbolic integration;
  * GENO limits: linear data give chi = 1 (blend exact); a step gives chi << 1.
"""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
import sympy as sp
import torch

from oracle import oracle as O
from paper_2508_08965_amd import workloads as W

mp.mp.dps = 40


def _basis():
    mi = []
    for deg in range(1, 5):
        for d0 in range(deg, -1, -1):
            for d1 in range(deg - d0, -1, -1):
                mi.append((d0, d1, deg - d0 - d1))
    return mi


def test_multi_index_order():
    assert [tuple(x) for x in O.constants()["MI"]] == _basis()


def _mp_system():
    """Rows of eq. (compact-big-ref) on the standard stencil, 40 digits, with their weights."""
    mi = _basis()
    half = mp.mpf(1) / 2
    g = 1 / (2 * mp.sqrt(3))

    def I(n, a, b):
        return (mp.mpf(b) ** (n + 1) - mp.mpf(a) ** (n + 1)) / (n + 1)

    def mean_mono(d, o):
        v = mp.mpf(1)
        for q in range(3):
            v *= I(d[q], o[q] - half, o[q] + half) / mp.factorial(d[q])
        return v

    zero = (0, 0, 0)

    def avg_p(d, o):
        return mean_mono(d, o) - mean_mono(d, zero)

    def avg_dp(d, j, o):
        if d[j] == 0:
            return mp.mpf(0)
        e = list(d); e[j] -= 1
        return mean_mono(e, o)

    def val_p(d, x):
        v = mp.mpf(1)
        for q in range(3):
            v *= mp.mpf(x[q]) ** d[q] / mp.factorial(d[q])
        return v - mean_mono(d, zero)

    faces = []
    for m in range(6):
        o = [0, 0, 0]; o[m // 2] = 1 if m % 2 else -1
        faces.append(o)
    edges = []
    for p, (a, b, c) in enumerate([(0, 1, 2), (0, 2, 1), (1, 2, 0)]):
        for n in range(4):
            o = [0, 0, 0]; o[a] = 1 if n & 1 else -1; o[b] = 1 if n & 2 else -1
            t1 = [0, 0, 0]; t1[c] = 1
            t2 = [mp.mpf(x) / mp.sqrt(2) for x in o]
            edges.append((o, t1, t2))
    rows, w = [], []
    for o in faces:
        rows.append([avg_p(d, o) for d in mi]); w.append(1)
    for o, _, _ in edges:
        rows.append([avg_p(d, o) for d in mi]); w.append(1)
    for o in faces:
        for j in range(3):
            rows.append([avg_dp(d, j, o) for d in mi]); w.append(2)
    for o, t1, t2 in edges:
        rows.append([sum(t1[j] * avg_dp(d, j, o) for j in range(3)) for d in mi]); w.append(1)
        rows.append([sum(t2[j] * avg_dp(d, j, o) for j in range(3)) for d in mi]); w.append(1)
    for q in range(3):
        ta, tb = [t for t in range(3) if t != q]
        for k in range(4):
            x1 = [0, 0, 0]; x1[ta] = (2 * (k & 1) - 1) * g; x1[tb] = (2 * (k >> 1) - 1) * g
            x2 = list(x1); x1[q] = -half; x2[q] = half
            rows.append([val_p(d, x2) - val_p(d, x1) for d in mi]); w.append(3)
    return mp.matrix(rows), w


def test_R_matches_40_digit_null_space_solution():
    A, w = _mp_system()
    C = A[0:6, :]
    # null space of the exact rows via a 40-digit QR of C^T
    Qf, _ = mp.qr(C.T, mode="full")
    Z = Qf[:, 6:34]
    Cp = C.T * mp.inverse(C * C.T)          # right inverse for the constraint rows
    AL = A[6:72, :]
    WL = mp.diag([w[r] for r in range(6, 72)])
    M = (WL * AL * Z)
    N = M.T * M
    Ninv = mp.inverse(N)
    # a = Cp bC + Z y, y = N^-1 (WL AL Z)^T WL (bL - AL Cp bC)
    P = Z * Ninv * M.T * WL
    R = mp.matrix(34, 72)
    part_c = Cp - P * AL * Cp
    for i in range(34):
        for j in range(6):
            R[i, j] = part_c[i, j]
        for j in range(66):
            R[i, 6 + j] = P[i, j]
    Rn = np.array([[float(R[i, j]) for j in range(72)] for i in range(34)])
    Ro = O.constants()["R"]
    assert np.abs(Ro - Rn).max() <= 1e-13 * np.abs(Rn).max()
    # exact rows hold exactly: C R = [I 0]
    Cn = np.array([[float(C[i, j]) for j in range(34)] for i in range(6)])
    np.testing.assert_allclose(Cn @ Ro, np.hstack([np.eye(6), np.zeros((6, 66))]), atol=1e-13)


def _quartic(rng):
    terms = [(a, b, c) for a in range(5) for b in range(5) for c in range(5) if a + b + c <= 4]
    return {t: rng.normal() for t in terms}


def _pval(coef, x, y, z):
    s = 0.0
    for (a, b, c), v in coef.items():
        s = s + v * x ** a * y ** b * z ** c
    return s


def _pder(coef, x, y, z, j):
    s = 0.0
    for (a, b, c), v in coef.items():
        e = [a, b, c]
        if e[j] == 0:
            continue
        f = e[j]; e[j] -= 1
        s = s + v * f * x ** e[0] * y ** e[1] * z ** e[2]
    return s


@pytest.mark.parametrize("mesh", ["cartesian", "affine"])
def test_quartic_exactness_at_gauss_points(mesh):
    rng = np.random.default_rng(21)
    c1, c2 = _quartic(rng), _quartic(rng)
    n = (6, 5, 4)
    nodes = (W.cartesian_nodes(n, (0, 0, 0), (0.6, 0.5, 0.4)) if mesh == "cartesian"
             else W.skewed_nodes(n, period=0.5))

    def prim(x, y, z):
        one = torch.ones_like(x)
        return 2.0 + 0.1 * _pval(c1, x, y, z), 0 * one, 0 * one, 0 * one, 3.0 + 0.1 * _pval(c2, x, y, z)

    Q, G, L = W.initial_state(nodes, prim, 1.4)
    cells = np.array([37, 44, 75, 82])  # interior cells: the polynomial is not periodic
    out = O.recon(n, nodes.numpy(), O.params(linear=1), Q.numpy(), G.numpy(), L.numpy(), cells)
    cr = W._corners(nodes)
    g = 0.5 / math.sqrt(3)
    for m in range(6):
        q = m // 2
        ta, tb = [t for t in range(3) if t != q]
        for k in range(4):
            xi = [0.0, 0.0, 0.0]
            xi[q] = 0.5 if m % 2 else -0.5
            xi[ta] = (2 * (k & 1) - 1) * g
            xi[tb] = (2 * (k >> 1) - 1) * g
            X, _ = W._map(cr, xi)
            X = X.reshape(-1, 3)[cells]
            x, y, z = X[:, 0], X[:, 1], X[:, 2]
            np.testing.assert_allclose(out[:, 4 * m + k, 0, 0], (2.0 + 0.1 * _pval(c1, x, y, z)).numpy(),
                                       atol=1e-13)
            np.testing.assert_allclose(out[:, 4 * m + k, 4, 0], ((3.0 + 0.1 * _pval(c2, x, y, z)) / 0.4).numpy(),
                                       atol=1e-12)
            for j in range(3):
                np.testing.assert_allclose(out[:, 4 * m + k, 0, 1 + j], (0.1 * _pder(c1, x, y, z, j)).numpy(),
                                           atol=1e-12)
                np.testing.assert_allclose(out[:, 4 * m + k, 4, 1 + j], (0.25 * _pder(c2, x, y, z, j)).numpy(),
                                           atol=1e-11)


def test_gram_matrices_exact_integration():
    c = O.constants()
    rng = np.random.default_rng(5)
    x, y, z = sp.symbols("x y z")
    mi = _basis()
    hf = sp.Rational(1, 2)

    def mono(d):
        return x ** d[0] * y ** d[1] * z ** d[2] / (sp.factorial(d[0]) * sp.factorial(d[1]) * sp.factorial(d[2]))

    def cube(e):
        return sp.integrate(e, (x, -hf, hf), (y, -hf, hf), (z, -hf, hf))

    a = [Fraction(int(v), 7) for v in rng.integers(-9, 10, size=34)]
    P = sum(sp.Rational(ai.numerator, ai.denominator) * (mono(d) - cube(mono(d))) for ai, d in zip(a, mi))
    P = sp.expand(P)
    tot = {1: 0, 2: 0, 3: 0, 4: 0}
    for l0 in range(5):
        for l1 in range(5):
            for l2 in range(5):
                s = l0 + l1 + l2
                if 1 <= s <= 4:
                    D = sp.diff(P, x, l0, y, l1, z, l2) if s else P
                    tot[s] += cube(sp.expand(D * D))
    av = np.array([float(v) for v in a])
    ish = float(tot[1] + tot[2] + tot[3] + tot[4])
    isl = float(tot[1])
    ist = float(tot[2] + tot[3] + tot[4])
    assert av @ c["GH"] @ av == pytest.approx(ish, rel=1e-13)
    assert av @ c["GL"] @ av == pytest.approx(isl, rel=1e-13)
    assert av @ c["GT"] @ av == pytest.approx(ist, rel=1e-13)


def test_linear_data_give_chi_one_and_exact_blend():
    """IS^tau = 0 for linear data => alpha = 1 => chi = 1; every P_m^1 is the same linear field."""
    n = (5, 5, 5)
    nodes = W.skewed_nodes(n, period=1.0)

    def prim(x, y, z):
        one = torch.ones_like(x)
        return 1.0 + 0.3 * x - 0.2 * y + 0.1 * z, 0.2 * x + 0.1 * y, 0 * one, 0.05 * z, 4.0 * one

    Q, G, L = W.initial_state(nodes, prim, 1.4)
    cells = np.array([31, 62, 93])  # interior
    lin = O.recon(n, nodes.numpy(), O.params(linear=1), Q.numpy(), G.numpy(), L.numpy(), cells)
    nl = O.recon(n, nodes.numpy(), O.params(linear=0), Q.numpy(), G.numpy(), L.numpy(), cells)
    np.testing.assert_allclose(nl, lin, rtol=1e-12, atol=1e-12)


def test_step_data_switch_to_low_order():
    """Across a jump the nonlinear values stay within the data range (ENO property)."""
    n = (8, 1, 1)
    nodes = W.cartesian_nodes(n, (0, 0, 0), (1.0, 0.125, 0.125))

    def prim(x, y, z):
        one = torch.ones_like(x)
        rho = torch.where(x < 0.5, one, 0.1 * one)
        return rho, 0 * one, 0 * one, 0 * one, one

    Q, G, L = W.initial_state(nodes, prim, 1.4)
    cells = np.array([3, 4])
    lin = O.recon(n, nodes.numpy(), O.params(linear=1), Q.numpy(), G.numpy(), L.numpy(), cells)
    nl = O.recon(n, nodes.numpy(), O.params(linear=0), Q.numpy(), G.numpy(), L.numpy(), cells)
    rho_nl = nl[:, :, 0, 0]
    rho_lin = lin[:, :, 0, 0]
    over_lin = max(rho_lin.max() - 1.0, 0.1 - rho_lin.min())
    over_nl = max(rho_nl.max() - 1.0, 0.1 - rho_nl.min(), 0.0)
    assert over_lin > 0.05                      # the quartic overshoots at the jump
    assert over_nl < 0.01 and over_nl < 0.1 * over_lin
