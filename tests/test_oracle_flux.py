"""Pins of the oracle's gas-kinetic flux (Sec. 2, eq. (flux), time linearisation,
eqs. (deri-t-f), (deri-t-q); collision times of Sec. 5).

None of these re-types the oracle's formulas:
  * uniform state  -> Euler flux, zero time derivative (closed form);
  * continuous data, any tau -> Navier-Stokes flux with mu = tau p, the BGK bulk
    viscosity and kappa = c_p mu / Pr (Chapman-Enskog; textbook NS flux written here);
  * tau = 0, continuous data -> F_t = dF_Euler/dQ . Q_t with Q_t = -div F_Euler
    (finite-difference Jacobian of the textbook Euler flux);
  * mirror symmetry (swap sides, flip normal);
  * discontinuous data -> brute-force quadrature in velocity space and time of the
    distribution of eq. (flux), with slopes from 5x5 solves of quadrature moment matrices.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

GAM = 1.4
K = (5.0 - 3.0 * GAM) / (GAM - 1.0)


def cons(rho, u, p):
    u = np.asarray(u, float)
    return np.array([rho, rho * u[0], rho * u[1], rho * u[2], p / (GAM - 1) + 0.5 * rho * u @ u])


def prim(q):
    rho = q[0]
    u = q[1:4] / rho
    p = (GAM - 1) * (q[4] - 0.5 * rho * u @ u)
    return rho, u, p


def euler_flux(q, n):
    rho, u, p = prim(q)
    un = u @ n
    return np.array([rho * un, q[1] * un + p * n[0], q[2] * un + p * n[1], q[3] * un + p * n[2], (q[4] + p) * un])


def ns_viscous_flux(q, g, n, mu, Pr):
    """Textbook NS viscous + heat flux (to be subtracted from the Euler flux).
    g[v][j] = d Q_v / d x_j.  Stress with the BGK bulk viscosity: trace factor 2/(K+3)."""
    rho, u, p = prim(q)
    T = p / rho
    du = np.array([[(g[1 + i][j] - u[i] * g[0][j]) / rho for j in range(3)] for i in range(3)])
    dp = np.array([(GAM - 1) * (g[4][j] - sum(u[i] * g[1 + i][j] for i in range(3)) + 0.5 * (u @ u) * g[0][j])
                   for j in range(3)])
    dT = (dp - T * np.array([g[0][j] for j in range(3)])) / rho
    div = np.trace(du)
    sig = mu * (du + du.T - 2.0 / (K + 3.0) * div * np.eye(3))
    cp = GAM / (GAM - 1)
    qh = -cp * mu / Pr * dT
    sn = sig @ n
    return np.array([0.0, sn[0], sn[1], sn[2], u @ sn - qh @ n])


def rand_state(rng):
    rho = rng.uniform(0.5, 2.0)
    u = rng.uniform(-0.8, 0.8, 3)
    p = rng.uniform(0.5, 2.0)
    return cons(rho, u, p)


def rand_normal(rng):
    n = rng.normal(size=3)
    return n / np.linalg.norm(n)


def test_uniform_state_gives_euler_flux():
    rng = np.random.default_rng(3)
    for mode in [dict(tau_zero=1), dict(), dict(viscous=1, mu0=0.01, Pr=0.72, prandtl_fix=1)]:
        prm = O.params(**mode)
        npts = 20
        q = np.array([rand_state(rng) for _ in range(npts)])
        g = np.zeros((npts, 5, 3))
        nrm = np.array([rand_normal(rng) for _ in range(npts)])
        st, F, Ft, S = O.flux(prm, q, g, q, g, nrm, 0.01)
        assert st == 0
        for t in range(npts):
            np.testing.assert_allclose(F[t], euler_flux(q[t], nrm[t]), rtol=1e-13, atol=1e-13)
            np.testing.assert_allclose(Ft[t], 0.0, atol=1e-11)
            for s in (0, 2):
                np.testing.assert_allclose(S[t, s], q[t], rtol=1e-13, atol=1e-13)
                np.testing.assert_allclose(S[t, s + 1], 0.0, atol=1e-11)


@pytest.mark.parametrize("prandtl", [False, True])
def test_continuous_data_gives_navier_stokes_flux(prandtl):
    """Chapman-Enskog limit: f = g0 [1 - tau (a.u + A) + t A] exactly for continuous data."""
    rng = np.random.default_rng(5)
    mu, Pr = 0.02, 0.72
    prm = O.params(viscous=1, visc_law=0, mu0=mu, Pr=Pr if prandtl else 1.0, prandtl_fix=int(prandtl))
    npts = 25
    q = np.array([rand_state(rng) for _ in range(npts)])
    g = rng.normal(scale=0.5, size=(npts, 5, 3))
    nrm = np.array([rand_normal(rng) for _ in range(npts)])
    st, F, Ft, S = O.flux(prm, q, g, q, g, nrm, 0.013)
    assert st == 0
    for t in range(npts):
        ref = euler_flux(q[t], nrm[t]) - ns_viscous_flux(q[t], g[t], nrm[t], mu, Pr if prandtl else 1.0)
        np.testing.assert_allclose(F[t], ref, rtol=1e-11, atol=1e-12)
        # interface state equals the continuous state; its time derivative is the Euler one
        np.testing.assert_allclose(S[t, 0], q[t], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(S[t, 2], q[t], rtol=1e-12, atol=1e-12)


def _div_euler(q, g):
    """-div F_Euler from gradients via a central-difference Jacobian of the Euler flux."""
    qt = np.zeros(5)
    for j in range(3):
        e = np.zeros(3); e[j] = 1.0
        Jm = np.zeros((5, 5))
        for v in range(5):
            h = 1e-6 * max(1.0, abs(q[v]))
            dq = np.zeros(5); dq[v] = h
            Jm[:, v] = (euler_flux(q + dq, e) - euler_flux(q - dq, e)) / (2 * h)
        qt -= Jm @ g[:, j]
    return qt


def test_tau_zero_time_derivative_is_euler_lax_wendroff():
    rng = np.random.default_rng(7)
    prm = O.params(tau_zero=1)
    npts = 15
    q = np.array([rand_state(rng) for _ in range(npts)])
    g = rng.normal(scale=0.3, size=(npts, 5, 3))
    nrm = np.array([rand_normal(rng) for _ in range(npts)])
    st, F, Ft, S = O.flux(prm, q, g, q, g, nrm, 0.02)
    assert st == 0
    for t in range(npts):
        qt = _div_euler(q[t], g[t])
        Jn = np.zeros((5, 5))
        for v in range(5):
            h = 1e-6 * max(1.0, abs(q[t][v]))
            dq = np.zeros(5); dq[v] = h
            Jn[:, v] = (euler_flux(q[t] + dq, nrm[t]) - euler_flux(q[t] - dq, nrm[t])) / (2 * h)
        np.testing.assert_allclose(F[t], euler_flux(q[t], nrm[t]), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(Ft[t], Jn @ qt, rtol=1e-7, atol=1e-7)
        np.testing.assert_allclose(S[t, 1], qt, rtol=1e-7, atol=1e-7)
        np.testing.assert_allclose(S[t, 3], qt, rtol=1e-7, atol=1e-7)


def test_mirror_symmetry():
    rng = np.random.default_rng(11)
    for mode in [dict(), dict(viscous=1, mu0=0.01, Pr=0.72, prandtl_fix=1), dict(tau_zero=1)]:
        prm = O.params(**mode)
        npts = 20
        ql = np.array([rand_state(rng) for _ in range(npts)])
        qr = np.array([rand_state(rng) for _ in range(npts)])
        gl = rng.normal(scale=0.3, size=(npts, 5, 3))
        gr = rng.normal(scale=0.3, size=(npts, 5, 3))
        nrm = np.array([rand_normal(rng) for _ in range(npts)])
        st, F, Ft, S = O.flux(prm, ql, gl, qr, gr, nrm, 0.01)
        st2, F2, Ft2, S2 = O.flux(prm, qr, gr, ql, gl, -nrm, 0.01)
        assert st == 0 and st2 == 0
        np.testing.assert_allclose(F2, -F, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(Ft2, -Ft, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(S2[:, 0], S[:, 2], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(S2[:, 1], S[:, 3], rtol=1e-10, atol=1e-10)


def test_nonphysical_state_flagged():
    prm = O.params()
    q = cons(1.0, [0.1, 0, 0], 1.0)[None]
    bad = q.copy(); bad[0, 4] = 0.0  # negative pressure
    g = np.zeros((1, 5, 3))
    st, *_ = O.flux(prm, q, g, bad, g, np.array([[1.0, 0, 0]]), 0.01)
    assert st == O.ENONPHYS


# ---------------------------------------------------------------- brute-force quadrature
def _gl(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


class _Grid:
    """Tensor velocity grid; functions are quadratic polynomials in s = xi^2 with grid coefficients."""

    def __init__(self, lo, hi, nu=80, nv=72):
        ul, wl = _gl(nu, lo[0], 0.0)
        ur, wr = _gl(nu, 0.0, hi[0])
        self.u = np.concatenate([ul, ur])
        self.wu = np.concatenate([wl, wr])
        self.v, self.wv = _gl(nv, lo[1], hi[1])
        self.w, self.ww = _gl(nv, lo[2], hi[2])
        self.U, self.V, self.W = np.meshgrid(self.u, self.v, self.w, indexing="ij")
        self.Wt = self.wu[:, None, None] * self.wv[None, :, None] * self.ww[None, None, :]


def _maxw(gd, rho, u, lam):
    e = (gd.U - u[0]) ** 2 + (gd.V - u[1]) ** 2 + (gd.W - u[2]) ** 2
    return rho * (lam / math.pi) ** 1.5 * np.exp(-lam * e)


def _psi(gd):
    """psi as [5] list of (c0, c1, c2) polynomials in s = xi^2."""
    z = np.zeros_like(gd.U)
    one = np.ones_like(gd.U)
    return [(one, z, z), (gd.U, z, z), (gd.V, z, z), (gd.W, z, z),
            (0.5 * (gd.U ** 2 + gd.V ** 2 + gd.W ** 2), 0.5 * one, z)]


def _mul(a, b):
    c0 = a[0] * b[0]
    c1 = a[0] * b[1] + a[1] * b[0]
    c2 = a[0] * b[2] + a[1] * b[1] + a[2] * b[0]
    assert np.all(a[2] * b[1] + a[1] * b[2] == 0) and np.all(a[2] * b[2] == 0)
    return (c0, c1, c2)


def _lin(coefs, polys):
    out = [0.0, 0.0, 0.0]
    for c, p in zip(coefs, polys):
        for i in range(3):
            out[i] = out[i] + c * p[i]
    return tuple(np.broadcast_to(o, polys[0][0].shape) * 1.0 for o in out)


def _integrate(gd, density, poly, lam, mask=None):
    """int poly * density dXi with the internal-DOF Gaussian of inverse temperature lam."""
    xs1, xs2 = K / (2 * lam), K * (K + 2) / (4 * lam * lam)
    f = (poly[0] + poly[1] * xs1 + poly[2] * xs2) * density * gd.Wt
    if mask is not None:
        f = f * mask
    return f.sum()


def _brute_flux(ql, gl, qr, gr, dt, tau):
    """Flux, time derivative and interface state/derivative from the distribution of eq. (flux),
    with normal (1,0,0) and everything obtained by quadrature and dense 5x5 solves."""
    rl, ul, pl = prim(ql)
    rr, ur, pr = prim(qr)
    laml, lamr = rl / (2 * pl), rr / (2 * pr)
    spread = 6.5 / math.sqrt(min(laml, lamr))
    lo = [min(ul[i], ur[i]) - spread for i in range(3)]
    hi = [max(ul[i], ur[i]) + spread for i in range(3)]
    gd = _Grid(lo, hi)
    ps = _psi(gd)
    pos = (gd.U > 0).astype(float)
    neg = 1.0 - pos

    def moments(density, lam, poly, mask=None):
        return np.array([_integrate(gd, density, _mul(poly, ps[a]), lam, mask) for a in range(5)])

    def mmat(density, lam, rho):
        return np.array([[_integrate(gd, density, _mul(ps[a], ps[b]), lam) / rho for b in range(5)]
                         for a in range(5)])

    one = (np.ones_like(gd.U), np.zeros_like(gd.U), np.zeros_like(gd.U))
    gL, gR = _maxw(gd, rl, ul, laml), _maxw(gd, rr, ur, lamr)
    ML, MR = mmat(gL, laml, rl), mmat(gR, lamr, rr)
    aL = [np.linalg.solve(ML, gl[:, j] / rl) for j in range(3)]
    aR = [np.linalg.solve(MR, gr[:, j] / rr) for j in range(3)]
    vel = [ps[1], ps[2], ps[3]]

    def slope_poly(a3):
        return _lin([1.0, 1.0, 1.0], [_mul(_lin(a3[j], ps), vel[j]) for j in range(3)])

    sL, sR = slope_poly(aL), slope_poly(aR)
    AL = np.linalg.solve(ML, -moments(gL, laml, sL) / rl)
    AR = np.linalg.solve(MR, -moments(gR, lamr, sR) / rr)
    W0 = moments(gL, laml, one, pos) + moments(gR, lamr, one, neg)
    r0, u0, p0 = prim(W0)
    lam0 = r0 / (2 * p0)
    g0 = _maxw(gd, r0, u0, lam0)
    M0 = mmat(g0, lam0, r0)
    dW0 = [moments(gL, laml, _lin(aL[j], ps), pos) + moments(gR, lamr, _lin(aR[j], ps), neg) for j in range(3)]
    ab = [np.linalg.solve(M0, dW0[j] / r0) for j in range(3)]
    s0 = slope_poly(ab)
    Ab = np.linalg.solve(M0, -moments(g0, lam0, s0) / r0)
    pA0, pAL, pAR = _lin(Ab, ps), _lin(AL, ps), _lin(AR, ps)

    # f(t) = sum_i c_i(t) phi_i(u): velocity moments of each phi_i by quadrature, then the
    # time integrals of the scalar coefficients c_i(t) of eq. (flux) by Gauss-Legendre in t
    parts = [(g0, lam0, one, None), (g0, lam0, s0, None), (g0, lam0, pA0, None),
             (gL, laml, one, pos), (gL, laml, sL, pos), (gL, laml, pAL, pos),
             (gR, lamr, one, neg), (gR, lamr, sR, neg), (gR, lamr, pAR, neg)]

    def coefs(t):
        e = math.exp(-t / tau) if tau > 0 else 0.0
        c_sl = ((t + tau) * e - tau) if tau > 0 else 0.0
        c_A = (t - tau + tau * e) if tau > 0 else t
        side = [e, -(tau + t) * e, -tau * e]
        return [1.0 - e, c_sl, c_A] + side + side

    def fbar(T, weight):
        ts, wts = _gl(64, 0.0, T)
        cbar = np.zeros(9)
        for t, wt in zip(ts, wts):
            cbar += wt * np.array(coefs(t))
        acc = np.zeros(5)
        for c, (dens, lam, poly, mask) in zip(cbar, parts):
            acc += c * moments(dens, lam, _mul(poly, weight), mask)
        return acc

    Fb1, Fb2 = fbar(dt, ps[1]), fbar(dt / 2, ps[1])
    Wb1, Wb2 = fbar(dt, one), fbar(dt / 2, one)
    F = (4 * Fb2 - Fb1) / dt
    Ft = 4 * (Fb1 - 2 * Fb2) / dt ** 2
    Wn = (4 * Wb2 - Wb1) / dt
    Wt = 4 * (Wb1 - 2 * Wb2) / dt ** 2
    # time derivative of the moments of each side's own Maxwellian evolution g_k (1 + A^k t):
    # int psi A^k g_k over all velocities, which the compatibility condition makes equal to
    # minus the moments of the slope term (a^k . u) g_k; taken here by quadrature of the latter
    dWl = -moments(gL, laml, sL)
    dWr = -moments(gR, lamr, sR)
    return F, Ft, Wn, Wt, dWl, dWr


@pytest.mark.parametrize("mode", ["inviscid", "tau_zero"])
def test_discontinuous_flux_against_velocity_space_quadrature(mode):
    rng = np.random.default_rng(13 if mode == "inviscid" else 17)
    dt = 0.02
    prm = O.params(tau_zero=1) if mode == "tau_zero" else O.params()
    for _ in range(3):
        ql = cons(rng.uniform(0.6, 1.5), rng.uniform(-0.5, 0.5, 3), rng.uniform(0.6, 1.5))
        qr = cons(rng.uniform(0.6, 1.5), rng.uniform(-0.5, 0.5, 3), rng.uniform(0.6, 1.5))
        gl = rng.normal(scale=0.4, size=(5, 3))
        gr = rng.normal(scale=0.4, size=(5, 3))
        st, F, Ft, S = O.flux(prm, ql[None], gl[None], qr[None], gr[None], np.array([[1.0, 0.0, 0.0]]), dt)
        assert st == 0
        pl, pr = prim(ql)[2], prim(qr)[2]
        tau = 0.0 if mode == "tau_zero" else (0.05 * dt + 5.0 * abs((pl - pr) / (pl + pr)) * dt)
        Fb, Ftb, Wn, Wt, dWl, dWr = _brute_flux(ql, gl, qr, gr, dt, tau)
        np.testing.assert_allclose(F[0], Fb, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(Ft[0], Ftb, rtol=1e-7, atol=1e-7 * np.abs(Ftb).max())
        e0 = 0.0 if tau == 0 else math.exp(-dt / tau)
        if mode == "inviscid":
            assert e0 > 0.05  # the one-sided terms carry real weight in these cases
        # one-sided interface values and their time derivatives (section "Temporal
        # discretization"): Q^k = (1 - e0) W(t) + e0 W^k, dQ^k/dt = (1 - e0) W_t + e0 dW^k/dt
        np.testing.assert_allclose(S[0, 0], (1 - e0) * Wn + e0 * ql, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(S[0, 2], (1 - e0) * Wn + e0 * qr, rtol=1e-9, atol=1e-9)
        for k, dW in ((1, dWl), (3, dWr)):
            want = (1 - e0) * Wt + e0 * dW
            np.testing.assert_allclose(S[0, k], want, rtol=1e-7, atol=1e-7 * np.abs(want).max())
