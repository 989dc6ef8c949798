"""Pins of the oracle's wall sides (symmetry planes and no-slip adiabatic walls).

Ghost data behind a wall are the mirror images of the cells inside (value and cell-averaged
gradient), and a wall face takes the GKS flux between the interior side and its mirror image.
These are pinned against what does not depend on that code:
  * a block with symmetry planes on its sides is the first octant of the periodic box of twice
    its size, when the initial field is mirror-symmetric (the Taylor-Green vortex is, about
    x, y, z = 0 and pi) and the mesh spacing is mirror-symmetric about the sides (stretched
    Cartesian nodes); the periodic oracle is pinned elsewhere, so the wall run must reproduce it
    to rounding, cell by cell, for Q, grad Q and the line derivatives;
  * a parallel shear flow u(y) between no-slip walls is the half of the periodic flow whose
    velocity is odd about the walls: for a flow independent of x and z the point inversion
    through the wall line, a symmetry of the equations, acts as reflecting y and reversing every
    velocity component.  The discrete flow is uniform in x and z only in its cell data: the
    polynomial reconstructed from them is even, not constant, in x and z, so the x- and
    z-derivatives at the Gauss points are odd; the wall pairs a Gauss point with itself where the
    point inversion pairs it with the opposite one.  The two agree to that truncation effect
    (6e-7 of U after six steps at 8 cells), while a ghost with the wrong sign of u, or the other
    wall type, misses by 4e-2 of U;
  * the shear wave's decay against the closed form exp(-nu pi^2 t / H^2) of the equations, for
    both wall types (sin profile between no-slip walls, cos profile between symmetry planes);
  * mass and total energy are conserved with walls on every side (the wall fluxes of both vanish
    by the mirror symmetry of the kinetic flux), and a gas at rest stays at rest;
  * sides that do not pair, or wall sides that are not planes normal to their axis, are refused.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2508_08965_amd import workloads as W

GAM = 1.4


def _state(nodes, field):
    Q, G, L = W.initial_state(nodes, field, GAM)
    return Q.numpy(), G.numpy(), L.numpy()


def _octant(a, dims_big, dims):
    """Cells with i, j, k below dims of an array [..., N_big] on the block dims_big."""
    nx, ny, nz = dims_big
    lead = a.shape[:-1]
    b = a.reshape(lead + (nz, ny, nx))[..., : dims[2], : dims[1], : dims[0]]
    return b.reshape(lead + (-1,))


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _tgv_prm(bc, Ma=0.3, linear=0):
    p0 = 1.0 / (GAM * Ma * Ma)
    return O.params(viscous=1, visc_law=1, mu0=1.0 / 1600, T_ref=p0, S_suth=p0 * 110.4 / 288.15, Pr=0.7,
                    prandtl_fix=1, linear=linear, bc=bc)


@pytest.mark.parametrize("linear", [0, 1])
def test_symmetry_planes_reproduce_the_doubled_periodic_taylor_green_vortex(linear):
    m = (6, 5, 4)
    dims, big = m, tuple(2 * x for x in m)
    nodes = W.stretched_nodes(dims, cells_per_half=m)
    nodes_big = W.stretched_nodes(big, cells_per_half=m)
    # the block's nodes are the first octant of the doubled periodic box's nodes
    assert np.array_equal(nodes.numpy(), nodes_big.numpy()[: m[2] + 1, : m[1] + 1, : m[0] + 1])
    f = W.taylor_green(Ma=0.3)
    Q, G, L = _state(nodes, f)
    Qb, Gb, Lb = _state(nodes_big, f)
    wall = _tgv_prm((1,) * 6, linear=linear)
    per = _tgv_prm((0,) * 6, linear=linear)
    dt = 0.5 * O.cfl_dt(big, nodes_big.numpy(), per, Qb)
    st, Qw, Gw, Lw, _, _ = O.run(dims, nodes.numpy(), wall, Q, G, L, 3, dt=dt)
    assert st == 0
    st, Qp, Gp, Lp, _, _ = O.run(big, nodes_big.numpy(), per, Qb, Gb, Lb, 3, dt=dt)
    assert st == 0
    assert _rel(Qw, _octant(Qp, big, dims)) < 1e-13
    assert _rel(Gw, _octant(Gp, big, dims)) < 1e-11
    assert _rel(Lw, _octant(Lp, big, dims)) < 1e-11
    # the flow moved: the comparison is not of two unchanged states
    assert _rel(Qw, Q) > 1e-6


def _shear_case(mode, ny, H=1.0, U=0.05, mu0=0.01):
    lx = 0.25
    dims = (2, ny, 2)
    nodes = W.stretched_nodes(dims, half=(lx, H, lx), cells_per_half=dims, amp=(0.0, 0.08, 0.0))
    prm = dict(viscous=1, visc_law=0, mu0=mu0, Pr=1.0)
    return dims, nodes, W.shear_wave(U=U, H=H, mode=mode), prm


def test_noslip_walls_reproduce_the_doubled_periodic_shear_flow():
    dims, nodes, f, prm = _shear_case("sin", 8)
    big = (2, 16, 2)
    nodes_big = W.stretched_nodes(big, half=(0.25, 1.0, 0.25), cells_per_half=dims, amp=(0.0, 0.08, 0.0))
    Q, G, L = _state(nodes, f)
    Qb, Gb, Lb = _state(nodes_big, f)
    per = O.params(**prm)
    dt = O.cfl_dt(big, nodes_big.numpy(), per, Qb)
    st, Qp, Gp, Lp, _, _ = O.run(big, nodes_big.numpy(), per, Qb, Gb, Lb, 6, dt=dt)
    assert st == 0
    Qo, Go, Lo = (_octant(a, big, dims) for a in (Qp, Gp, Lp))
    diffs = {}
    for bc in (2, 1):
        wall = O.params(bc=(0, 0, bc, bc, 0, 0), **prm)
        st, Qw, Gw, Lw, _, _ = O.run(dims, nodes.numpy(), wall, Q, G, L, 6, dt=dt)
        assert st == 0
        diffs[bc] = [np.max(np.abs(a - b)) for a, b in ((Qw, Qo), (Gw, Go), (Lw, Lo))]
    # U = 0.05: |rho u| up to 5e-2, |grad rho u| up to 0.16, |L| up to 2.3e-2
    assert diffs[2][0] < 1e-6 and diffs[2][1] < 1e-5 and diffs[2][2] < 5e-6, diffs[2]
    assert diffs[1][0] > 1e-3 and diffs[1][1] > 1e-2 and diffs[1][2] > 1e-3, diffs[1]


@pytest.mark.parametrize("mode,bc", [("sin", 2), ("cos", 1)])
def test_shear_wave_decays_at_the_viscous_rate_between_walls(mode, bc):
    H, U, mu0 = 1.0, 0.05, 0.01
    dims, nodes, f, prm = _shear_case(mode, 12, H=H, U=U, mu0=mu0)
    Q, G, L = _state(nodes, f)
    P = O.params(bc=(0, 0, bc, bc, 0, 0), **prm)
    st, Qe, _, _, _, t = O.run(dims, nodes.numpy(), P, Q, G, L, 40)
    assert st == 0 and t > 0.5
    decay = math.exp(-mu0 * math.pi ** 2 * t / H ** 2)
    # cell averages of rho u against the decayed initial profile (rho = 1 initially)
    rel = np.max(np.abs(Qe[1] - decay * Q[1])) / (U * decay)
    assert rel < 2e-3, rel
    # the other wall type would not fit: its profile decays at another rate or not at all
    assert 1.0 - decay > 0.03


@pytest.mark.parametrize("bc", [1, 2])
def test_walls_on_every_side_conserve_mass_and_energy(bc):
    dims = (6, 6, 6)
    nodes = W.wall_perturbed_nodes(dims)
    Q, G, L = _state(nodes, W.taylor_green(Ma=0.3))
    P = _tgv_prm((bc,) * 6)
    vol = O.metrics(dims, nodes.numpy())["vol"]
    st, Qe, _, _, _, _ = O.run(dims, nodes.numpy(), P, Q, G, L, 5)
    assert st == 0
    for v in (0, 4):
        m0, m1 = np.dot(vol, Q[v]), np.dot(vol, Qe[v])
        assert abs(m1 - m0) <= 1e-13 * abs(m0), (v, m1 - m0)
    assert _rel(Qe, Q) > 1e-6


def test_gas_at_rest_stays_at_rest_between_noslip_walls():
    dims = (4, 5, 3)
    nodes = W.wall_perturbed_nodes(dims)
    Q, G, L = _state(nodes, W.uniform(rho=1.2, u=0.0, v=0.0, w=0.0, p=0.9))
    P = O.params(viscous=1, mu0=0.01, bc=(2,) * 6)
    st, Qe, Ge, Le, _, _ = O.run(dims, nodes.numpy(), P, Q, G, L, 4)
    assert st == 0
    assert np.max(np.abs(Qe - Q)) < 1e-14
    assert np.max(np.abs(Ge)) < 1e-12 and np.max(np.abs(Le)) < 1e-12


@pytest.mark.parametrize("bc", [(1, 0, 0, 0, 0, 0), (0, 0, 0, 2, 0, 0), (0, 0, 3, 0, 0, 0), (5, 5, 0, 0, 0, 0), (-1, -1, 0, 0, 0, 0)])
def test_unpaired_or_unknown_sides_are_refused(bc):
    dims = (4, 4, 4)
    nodes = W.cartesian_nodes(dims)
    Q, G, L = _state(nodes, W.uniform())
    with pytest.raises(ValueError):
        O.cfl_dt(dims, nodes.numpy(), O.params(bc=bc), Q)


def test_walls_on_sides_that_are_not_axis_planes_are_refused():
    dims = (6, 6, 6)
    nodes = W.skewed_nodes(dims)  # its sides are planes, but not normal to the axes
    Q, G, L = _state(nodes, W.uniform())
    with pytest.raises(ValueError):
        O.cfl_dt(dims, nodes.numpy(), O.params(bc=(1, 1, 0, 0, 0, 0)), Q)
    # the same mesh is accepted with periodic sides
    assert O.cfl_dt(dims, nodes.numpy(), O.params(), Q) > 0


@pytest.mark.parametrize("bc", [(1, 1, 2, 2, 1, 1), (2, 2, 1, 1, 0, 0)])
def test_sampled_stage1_with_walls_matches_the_whole_mesh_stage(bc):
    """The per-cell stage-1 entry point (used for sampled parity at full size) against a stage
    over the whole mesh, for corner, edge, face and interior cells."""
    dims = (7, 6, 5)
    nodes = W.wall_perturbed_nodes(dims)
    if bc[4] == 0:
        nodes[..., 2] *= 2.0  # periodic z spans the field's period
    Q, G, L = _state(nodes, W.taylor_green(Ma=0.3))
    P = _tgv_prm(bc)
    dt = 0.5 * O.cfl_dt(dims, nodes.numpy(), P, Q)
    N = Q.shape[1]
    cells = np.array([0, dims[0] - 1, N - 1, N - dims[0], 3 + 7 * 2 + 42 * 2, 7 * 3, 42 * 4 + 6, 5], dtype=np.int64)
    st, oq, og, ol = O.stage1_cells(dims, nodes.numpy(), P, dt, Q, G, L, cells)
    assert st == 0
    Qs, Gs, Ls = Q.copy(), G.copy(), L.copy()
    stash = np.zeros((90, N))
    assert O.stage(dims, nodes.numpy(), P, 1, dt, Qs, Gs, Ls, stash) == 0
    assert np.max(np.abs(oq - Qs[:, cells].T)) <= 1e-14 * np.max(np.abs(Qs))
    assert np.max(np.abs(og - Gs[:, :, cells].transpose(2, 0, 1))) <= 1e-12 * np.max(np.abs(Gs))
    assert np.max(np.abs(ol - Ls[:, :, cells].transpose(2, 0, 1))) <= 1e-12 * np.max(np.abs(Ls))


# ---- far-field sides (reading D27): ghost = the prescribed far-field state, uniform ----------

def _far_state(rho=1.2, u=(0.3, -0.2, 0.1), p=0.9):
    e = p / (GAM - 1.0) + 0.5 * rho * sum(x * x for x in u)
    return rho, u, p, (rho, rho * u[0], rho * u[1], rho * u[2], e)


@pytest.mark.parametrize("bc,u", [((3,) * 6, (0.3, -0.2, 0.1)), ((3, 3, 1, 1, 0, 0), (0.3, 0.0, 0.1))])
def test_far_field_sides_preserve_their_free_stream(bc, u):
    """A uniform flow equal to the far-field state is a steady solution: far-field sides (and
    symmetry planes parallel to the flow) keep it to rounding on a curvilinear box."""
    dims = (6, 5, 4)
    nodes = W.wall_perturbed_nodes(dims)
    if bc[4] == 0:
        nodes[..., 2] *= 2.0
    rho, u, p, far = _far_state(u=u)
    Q, G, L = _state(nodes, W.uniform(rho=rho, u=u[0], v=u[1], w=u[2], p=p))
    P = O.params(viscous=1, mu0=0.01, bc=bc, far=far)
    st, Qe, Ge, Le, _, _ = O.run(dims, nodes.numpy(), P, Q, G, L, 4)
    assert st == 0
    assert np.max(np.abs(Qe - Q)) < 1e-13
    assert np.max(np.abs(Ge)) < 1e-11 and np.max(np.abs(Le)) < 1e-12


def _pulse_run(bc, n=64, t_end=1.2):
    """Gaussian acoustic pulse (linear: rho' = p'/c^2, u' = 0) at the centre of [0, 1] along x,
    one cell across in y and z (periodic); inviscid; returns max |p - p0| over the initial one."""
    dims = (n, 1, 1)
    h = 1.0 / n
    nodes = W.cartesian_nodes(dims, hi=(1.0, h, h))
    p0, rho0, amp = 1.0 / GAM, 1.0, 1e-3

    def f(x, y, z):
        g = amp * torch.exp(-((x - 0.5) / 0.05) ** 2)
        zero = torch.zeros_like(x)
        return rho0 + g, zero, zero, zero, p0 * (1.0 + GAM * g)
    Q, G, L = _state(nodes, f)
    far = (rho0, 0.0, 0.0, 0.0, p0 / (GAM - 1.0))
    P = O.params(bc=bc, far=far)
    press = lambda Qa: (GAM - 1.0) * (Qa[4] - 0.5 * (Qa[1] ** 2 + Qa[2] ** 2 + Qa[3] ** 2) / Qa[0])
    d0 = np.max(np.abs(press(Q) - p0))
    t, Qc, Gc, Lc = 0.0, Q, G, L
    while t < t_end:
        st, Qc, Gc, Lc, dt, dtt = O.run(dims, nodes.numpy(), P, Qc, Gc, Lc, 20)
        assert st == 0
        t += dtt
    return np.max(np.abs(press(Qc) - p0)) / d0


def test_acoustic_pulse_leaves_through_far_field_sides():
    """The two halves of the pulse reach the sides at t = 0.5 and have left by t = 1.2 (c = 1):
    far-field sides let them out (what stays is the reflection of the kinetic flux against the
    uniform far-field state), symmetry planes send them back."""
    far = _pulse_run((3, 3, 0, 0, 0, 0))
    wall = _pulse_run((1, 1, 0, 0, 0, 0))
    assert far < 0.01, far  # 1.5e-3 measured
    assert wall > 0.3, wall  # each reflected half carries half the amplitude: 0.46 measured


@pytest.mark.parametrize("far", [(0.0, 0, 0, 0, 2.5), (1.0, 0, 0, 0, 0.0), (1.0, 3.0, 0, 0, 2.5)])
def test_far_field_state_must_be_physical(far):
    dims = (4, 4, 4)
    nodes = W.cartesian_nodes(dims)
    Q, G, L = _state(nodes, W.uniform())
    with pytest.raises(ValueError):
        O.cfl_dt(dims, nodes.numpy(), O.params(bc=(3, 3, 0, 0, 0, 0), far=far), Q)
