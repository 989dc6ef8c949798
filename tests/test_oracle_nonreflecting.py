"""Pins of the oracle's non-reflecting sides (side type 4, reading D29).

At a non-reflecting side the stencil's ghost cells are the linear continuation of the cell
beside the side (its average plus its reference gradient times the one-cell offset along the
side's axis, its gradient unchanged), and the side's faces take the GKS flux between the
interior Gauss-point state and a boundary state from locally one-dimensional characteristics
(Riemann invariants u_n +- 2c/(gamma - 1): the outgoing one from the interior, the incoming one
from the far-field state; entropy and tangential velocity from the upwind side).  Pinned by:
  * the boundary state against the definition of the invariants, independently of the code's
    steps: the outgoing invariant of the state is the interior's, the incoming one the far
    field's, entropy and tangential velocity those of the upwind side;
  * an outgoing isentropic simple wave (its incoming invariant and entropy those of the far
    field) has itself as the boundary state, the far-field state likewise; supersonic outflow
    and inflow take the interior and the far-field state;
  * a linear field is reconstructed exactly in cells beside non-reflecting sides (the linear
    continuation is exact data for it; a far-field ghost is not);
  * a uniform flow equal to the far-field state is kept to rounding on a curvilinear box;
  * an acoustic pulse leaves through non-reflecting sides with a residual that falls with the
    mesh (second order), where the far-field side's does not.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_08965_amd import workloads as W

GAM = 1.4


def _cons(rho, u, p):
    u = np.asarray(u, dtype=float)
    return np.array([rho, *(rho * u), p / (GAM - 1.0) + 0.5 * rho * u @ u])


def _prim(q):
    rho, u = q[0], q[1:4] / q[0]
    p = (GAM - 1.0) * (q[4] - 0.5 * rho * u @ u)
    return rho, u, p


FAR = _cons(1.1, (0.2, -0.1, 0.05), 0.8)


def _prm(**kw):
    return O.params(far=tuple(FAR), **kw)


def _invariants(q, n):
    rho, u, p = _prim(q)
    c = math.sqrt(GAM * p / rho)
    un = u @ n
    return un + 2 * c / (GAM - 1), un - 2 * c / (GAM - 1), p / rho ** GAM, u - un * n


@pytest.mark.parametrize("un,seed", [(0.15, 1), (-0.12, 2), (0.02, 3), (-0.3, 4)])
def test_boundary_state_carries_the_invariants_of_its_upwind_sides(un, seed):
    rng = np.random.default_rng(seed)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    t = rng.normal(size=3)
    u = un * n + 0.2 * (t - (t @ n) * n)
    q = _cons(0.9 + 0.2 * rng.random(), u, 0.7 + 0.2 * rng.random())
    qb = O.nonreflecting_state(_prm(), q, n)
    out_b, in_b, s_b, ut_b = _invariants(qb, n)
    out_i, _, s_i, ut_i = _invariants(q, n)
    _, in_e, s_e, ut_e = _invariants(FAR, n)
    assert out_b == pytest.approx(out_i, rel=1e-13, abs=1e-13)
    assert in_b == pytest.approx(in_e, rel=1e-13, abs=1e-13)
    ub = qb[1:4] / qb[0]
    if ub @ n > 0:  # outflow through the side: entropy and tangential velocity of the interior
        assert s_b == pytest.approx(s_i, rel=1e-13)
        np.testing.assert_allclose(ut_b, ut_i, rtol=0, atol=1e-14)
    else:
        assert s_b == pytest.approx(s_e, rel=1e-13)
        np.testing.assert_allclose(ut_b, ut_e, rtol=0, atol=1e-14)


@pytest.mark.parametrize("du", [0.05, -0.05, 0.2])
def test_outgoing_simple_wave_and_far_field_are_their_own_boundary_state(du):
    n = np.array([0.0, 0.6, 0.8])
    rho_e, u_e, p_e = _prim(FAR)
    c_e = math.sqrt(GAM * p_e / rho_e)
    # the simple wave: same entropy and incoming invariant as the far field, u_n shifted by du
    c = c_e + 0.5 * (GAM - 1.0) * du
    rho = rho_e * (c * c / (c_e * c_e)) ** (1.0 / (GAM - 1.0))
    q = _cons(rho, u_e + du * n, rho * c * c / GAM)
    np.testing.assert_allclose(O.nonreflecting_state(_prm(), q, n), q, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(O.nonreflecting_state(_prm(), FAR, n), FAR, rtol=1e-14, atol=1e-14)


def test_supersonic_outflow_and_inflow():
    n = np.array([1.0, 0.0, 0.0])
    q_out = _cons(1.0, (2.0, 0.1, 0.0), 0.7)  # c = 0.99: u_n > c
    q_in = _cons(1.0, (-2.0, 0.1, 0.0), 0.7)
    np.testing.assert_array_equal(O.nonreflecting_state(_prm(), q_out, n), q_out)
    np.testing.assert_array_equal(O.nonreflecting_state(_prm(), q_in, n), FAR)


def _linear_field(x, y, z):
    import torch
    zero = torch.zeros_like(x)
    return 1.0 + 0.1 * x + 0.05 * y - 0.02 * z, zero, zero, zero, 1.0 + 0.2 * x - 0.1 * y + 0.03 * z


@pytest.mark.parametrize("bc,exact", [((4,) * 6, True), ((3,) * 6, False)])
def test_linear_field_is_reconstructed_exactly_beside_nonreflecting_sides(bc, exact):
    dims = (5, 4, 3)
    h = (0.3, 0.5, 0.7)
    nodes = W.cartesian_nodes(dims, hi=tuple(h[q] * dims[q] for q in range(3)))
    Q, G, L = (t.numpy() for t in W.initial_state(nodes, _linear_field, GAM))
    N = Q.shape[1]
    cells = np.arange(N)
    gp = O.recon(dims, nodes.numpy(), _prm(bc=bc), Q, G, L, cells)
    gq = 0.5 / math.sqrt(3.0)
    err = 0.0
    for c in cells:
        for u in range(6):
            q = u // 2
            for g in range(4):
                ta, tb = (gq if g & 1 else -gq), (gq if g & 2 else -gq)
                xi = [ta, ta if q == 0 else tb, tb]
                xi[q] = 0.5 if u & 1 else -0.5
                if q == 0:
                    xi = [xi[0], ta, tb]
                elif q == 1:
                    xi = [ta, xi[1], tb]
                else:
                    xi = [ta, tb, xi[2]]
                d = np.array([xi[r] * h[r] for r in range(3)])
                for v in (0, 4):
                    want = Q[v, c] + G[v, :, c] @ d
                    err = max(err, abs(gp[c, 4 * u + g, v, 0] - want),
                              np.max(np.abs(gp[c, 4 * u + g, v, 1:] - G[v, :, c])))
    if exact:
        assert err < 1e-13, err
    else:
        assert err > 1e-4, err  # a far-field ghost is not the field's continuation


@pytest.mark.parametrize("bc,far", [((4,) * 6, FAR), ((4, 4, 1, 1, 0, 0), _cons(1.1, (0.2, 0.0, 0.05), 0.8))])
def test_free_stream_kept_with_nonreflecting_sides(bc, far):
    """With non-reflecting sides alone, and with symmetry planes parallel to the flow."""
    dims = (6, 5, 4)
    nodes = W.wall_perturbed_nodes(dims)
    if bc[4] == 0:
        nodes[..., 2] *= 2.0
    rho, u, p = _prim(far)
    Q, G, L = (t.numpy() for t in W.initial_state(nodes, W.uniform(rho=rho, u=u[0], v=u[1], w=u[2], p=p), GAM))
    P = O.params(far=tuple(far), viscous=1, mu0=0.01, bc=bc)
    st, Qe, Ge, Le, _, _ = O.run(dims, nodes.numpy(), P, Q, G, L, 4)
    assert st == 0
    assert np.max(np.abs(Qe - Q)) < 1e-13
    assert np.max(np.abs(Ge)) < 1e-11 and np.max(np.abs(Le)) < 1e-12


def test_acoustic_pulse_leaves_and_its_reflection_falls_with_the_mesh():
    from test_oracle_walls import _pulse_run
    nr = [_pulse_run((4, 4, 0, 0, 0, 0), n=n) for n in (32, 64, 128)]
    far = [_pulse_run((3, 3, 0, 0, 0, 0), n=n) for n in (32, 128)]
    # measured 6.2e-4, 3.2e-4, 8.4e-5 against 1.2e-3 and 3.1e-3 for far-field sides
    assert nr[0] > nr[1] > nr[2] and nr[2] < 0.25 * nr[0], nr
    assert nr[2] < 0.05 * far[1], (nr, far)
    assert far[1] > far[0], far
