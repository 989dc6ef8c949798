"""The interface-state limiter of reading D28 (an addition to the paper for flows whose local
Mach number reaches ~3, where internal energy is a small part of the total): pins of the
oracle's closed form against brute force, and its effect on a whole run.

At a face Gauss point a cell's reconstructed state q (gradient g) is replaced by
qbar + theta (q - qbar) (gradient theta g), theta the largest value in [0, 1] that keeps the
density and pressure at or above eps times the cell average's own.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_08965_amd import workloads as W

GAM = 1.4
EPS = 1e-3


def prim_p(q):
    return (GAM - 1.0) * (q[..., 4] - 0.5 * (q[..., 1] ** 2 + q[..., 2] ** 2 + q[..., 3] ** 2) / q[..., 0])


def cons(rho, u, p):
    u = np.asarray(u, dtype=float)
    return np.concatenate([[rho], rho * u, [p / (GAM - 1.0) + 0.5 * rho * u @ u]])


def ok(z, qb):
    return z[0] >= EPS * qb[0] and prim_p(z) >= EPS * prim_p(qb)


def brute_theta(qb, q, n=20000):
    """Largest theta on a fine grid, then refined by bisection, with the segment state at or
    above both floors (every grid point up to it too: the admissible set is an interval)."""
    ts = np.linspace(0.0, 1.0, n + 1)
    good = np.array([ok(qb + t * (q - qb), qb) for t in ts])
    if good.all():
        return 1.0
    k = int(np.argmin(good))  # first failing grid point
    lo, hi = ts[k - 1], ts[k]
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if ok(qb + mid * (q - qb), qb):
            lo = mid
        else:
            hi = mid
    return lo


def random_cases(rng, n):
    qb, q = [], []
    for _ in range(n):
        rho, p = rng.uniform(0.3, 2.0), rng.uniform(0.3, 2.0)
        u = rng.uniform(-2.5, 2.5, 3)
        qb.append(cons(rho, u, p))
        # a Gauss-point state far from the average: large velocity change, density dip
        q.append(cons(rho * rng.uniform(-0.5, 1.5), u + rng.normal(scale=1.5, size=3), p * rng.uniform(-1.0, 1.5)))
    return np.array(qb), np.array(q)


def test_limiter_matches_brute_force_and_keeps_the_floor():
    rng = np.random.default_rng(28)
    qb, q = random_cases(rng, 300)
    g = rng.normal(size=(300, 5, 3))
    prm = O.params(positivity=1, pos_eps=EPS)
    ql, gl = O.positivity(prm, qb, q, g)
    active = 0
    for i in range(300):
        th = brute_theta(qb[i], q[i])
        if th >= 1.0:
            np.testing.assert_array_equal(ql[i], q[i])  # untouched where already physical
            np.testing.assert_array_equal(gl[i], g[i])
            continue
        active += 1
        want = qb[i] + th * (q[i] - qb[i])
        np.testing.assert_allclose(ql[i], want, rtol=1e-9, atol=1e-9 * np.abs(qb[i]).max())
        np.testing.assert_allclose(gl[i], th * g[i], rtol=1e-9, atol=1e-12)
        # at the floor: the binding bound holds with equality, the other with room
        r, p = ql[i][0] / (EPS * qb[i][0]), prim_p(ql[i]) / (EPS * prim_p(qb[i]))
        assert min(r, p) == pytest.approx(1.0, rel=1e-8)
        assert r >= 1.0 - 1e-9 and p >= 1.0 - 1e-9
    assert active > 100  # the cases do exercise the limiter


def test_limiter_density_and_pressure_bounds_separately():
    prm = O.params(positivity=1, pos_eps=EPS)
    qb = cons(1.0, (0.3, 0.0, 0.0), 1.0)[None]
    # density below the floor, pressure fine: theta from the linear density bound
    q = cons(-0.5, (0.3, 0.0, 0.0), 1.0)[None]
    ql, _ = O.positivity(prm, qb, q, np.zeros((1, 5, 3)))
    th = (1.0 - EPS) / (1.0 + 0.5)
    np.testing.assert_allclose(ql[0], qb[0] + th * (q[0] - qb[0]), rtol=1e-13)
    # a fast stream of the same total energy: pressure negative, density fine
    q = qb.copy()
    q[0, 1:4] = [2.5, 0.0, 0.0]
    ql, _ = O.positivity(prm, qb, q, np.zeros((1, 5, 3)))
    assert prim_p(ql[0]) == pytest.approx(EPS * prim_p(qb[0]), rel=1e-10)
    # a non-physical cell average: left alone (it is flagged elsewhere)
    bad = cons(1.0, (0.0, 0.0, 0.0), 1.0)[None]
    bad[0, 4] = -1.0
    ql, _ = O.positivity(prm, bad, q, np.zeros((1, 5, 3)))
    np.testing.assert_array_equal(ql, q)


def test_limiter_off_by_default_and_not_with_walls():
    n = (6, 5, 4)
    nodes = W.cartesian_nodes(n)
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    a = O.run(n, nodes.numpy(), O.params(), Q.numpy(), G.numpy(), L.numpy(), 2)
    b = O.run(n, nodes.numpy(), O.params(positivity=1), Q.numpy(), G.numpy(), L.numpy(), 2)
    for x, y in zip(a[1:4], b[1:4]):  # smooth subsonic flow: the limiter never acts
        np.testing.assert_array_equal(x, y)
    st = O.run(n, nodes.numpy(), O.params(positivity=1, bc=(1, 1, 0, 0, 0, 0)), Q.numpy(), G.numpy(), L.numpy(),
               1)[0]
    assert st == O.EINVAL


@pytest.mark.slow
def test_supersonic_turbulence_stays_physical_with_the_limiter():
    """Isotropic turbulence at Mt 1.0 (k0 8) on 32^3: the plain scheme meets a non-physical
    state once shocklets form; with the limiter the run reaches t = lambda / u' = 0.43."""
    n = (32, 32, 32)
    nodes = W.cartesian_nodes(n, hi=(2 * math.pi,) * 3)
    Q, G, L = W.initial_state(nodes, W.isotropic_turbulence(32, k0=8.0, Mt=1.0, seed=8967), GAM)
    T0 = 1.0 / GAM
    kw = dict(viscous=1, visc_law=1, mu0=1.44e-3, T_ref=T0, S_suth=T0 * 110.4 / 288.15, Pr=0.72, prandtl_fix=1)
    t_end = 0.25 / 0.5774

    def run(pos):
        q, g, l = Q.numpy(), G.numpy(), L.numpy()
        t = 0.0
        for _ in range(60):
            st, q, g, l, dt, _ = O.run(n, nodes.numpy(), O.params(positivity=pos, **kw), q, g, l, 1)
            if st:
                return st, t
            t += dt
            if t >= t_end:
                break
        return 0, t

    st, t = run(0)
    assert st == O.ENONPHYS and t < t_end
    st, t = run(1)
    assert st == 0 and t >= t_end
