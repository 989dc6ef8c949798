"""GPU parity of wall sides (symmetry planes, no-slip adiabatic walls) against the oracle.

The oracle's walls are pinned on the CPU (doubled periodic domain, viscous decay of a shear
wave, conservation).  Here the HIP path runs the same seeded inputs through the C ABI and is
compared element by element at the FP64 bar of the periodic parity tests: relative L2 1e-12
for Q, the oracle's measured rounding spread for G and L (tests/parity_bar.py).  Meshes span several reconstruction tiles with
a ragged tail; one block is one cell thick along a wall axis (both wall faces of a line in one
record); the curvilinear wall mesh keeps its sides planar.
"""
import math

import numpy as np
import pytest
import torch

import parity_bar as PB
from oracle import oracle as O
from paper_2508_08965_amd import workloads as W

pytestmark = pytest.mark.gpu

GAM = 1.4
TOL = 1e-12


def K():
    from paper_2508_08965_amd import cgks
    return cgks


def dev():
    return torch.device("cuda:0")


def rel_l2(a, b):
    a = a.detach().cpu().numpy() if torch.is_tensor(a) else a
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def assert_whole_run(Qd, Gd, Ld, ref, sp):
    Qo, Go, Lo = ref
    PB.assert_rel(Qd, Qo, "Q")
    PB.assert_spread_parity(Gd, Go, sp["G"], "G")
    PB.assert_spread_parity(Ld, Lo, sp["L"], "L")


def tgv_kw(Ma=0.3, bc=(0,) * 6):
    p0 = 1.0 / (GAM * Ma * Ma)
    return dict(viscous=1, visc_law=1, mu0=1.0 / 1600, T_ref=p0, S_suth=p0 * 110.4 / 288.15, Pr=0.72,
                prandtl_fix=1, bc=bc)


def run_gpu(dims_list, nodes_list, prm, Q, G, L, nsteps, dt=None):
    ctx = K().Context(dims_list, nodes_list, prm)
    Qd, Gd, Ld = Q.clone().to(dev()), G.clone().to(dev()), L.clone().to(dev())
    dtd = torch.zeros(1, dtype=torch.float64, device=dev())
    if dt is not None:
        dtd.fill_(dt)
    dts = []
    for _ in range(nsteps):
        K().cgks_step(ctx, Qd, Gd, Ld, dtd, use_cfl=dt is None)
        dts.append(dtd.item())
    torch.cuda.synchronize()
    st = K().cgks_check(ctx)
    ctx.close()
    return st, Qd, Gd, Ld, dts


CASES = {
    # name: (dims, mesh, bc)
    "symmetry_all_sides_stretched": ((20, 18, 16), "stretched", (1, 1, 1, 1, 1, 1)),
    "noslip_all_sides_curvilinear": ((20, 18, 16), "curved", (2, 2, 2, 2, 2, 2)),
    "mixed_sym_x_noslip_y_periodic_z": ((19, 17, 12), "curved_z2", (1, 1, 2, 2, 0, 0)),
    "one_cell_thick_wall_axis": ((24, 1, 20), "thin_y", (0, 0, 2, 2, 0, 0)),
}


def mesh(kind, dims):
    """Walls span [0, pi] (the Taylor-Green field is mirror-symmetric there); periodic axes span
    its period 2 pi."""
    if kind == "stretched":
        return W.stretched_nodes(dims, cells_per_half=dims)
    if kind == "curved":
        return W.wall_perturbed_nodes(dims)
    if kind == "curved_z2":
        n = W.wall_perturbed_nodes(dims)
        n[..., 2] *= 2.0  # z periodic on [0, 2 pi]; the x and y sides stay planes
        return n
    return W.stretched_nodes(dims, half=(2 * math.pi, math.pi, 2 * math.pi), cells_per_half=dims,
                             amp=(0.0, 0.1, 0.0))


@pytest.mark.parametrize("name", list(CASES))
def test_wall_parity_with_oracle(name):
    dims, kind, bc = CASES[name]
    print(f"walls case {name} dims {dims} bc {bc}", flush=True)
    nodes = mesh(kind, dims)
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    kw = tgv_kw(bc=bc)
    st, Qd, Gd, Ld, dts = run_gpu([dims], [nodes], K().default_params(**kw), Q, G, L, 4)
    assert st == (0, 0)
    ref, sp, dto = PB.oracle_run_pair(dims, nodes, O.params(**kw), Q, G, L, 4)
    assert dts[-1] == pytest.approx(dto, rel=1e-13)
    assert_whole_run(Qd, Gd, Ld, ref, sp)
    assert rel_l2(Qd, Q.numpy()) > 1e-7  # the state moved


@pytest.mark.parametrize("bc", [1, 2])
def test_walls_conserve_mass_and_energy_on_the_gpu(bc):
    dims = (24, 20, 16)
    nodes = W.wall_perturbed_nodes(dims)
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    ctx = K().Context([dims], [nodes], K().default_params(**tgv_kw(bc=(bc,) * 6)))
    vol = torch.zeros(ctx.ncells, dtype=torch.float64, device=dev())
    K().cgks_metrics(ctx, vol=vol)
    Qd, Gd, Ld = Q.clone().to(dev()), G.clone().to(dev()), L.clone().to(dev())
    dtd = torch.zeros(1, dtype=torch.float64, device=dev())
    m0 = (vol * Qd[0]).sum().item(), (vol * Qd[4]).sum().item()
    for _ in range(10):
        K().cgks_step(ctx, Qd, Gd, Ld, dtd, use_cfl=True)
    m1 = (vol * Qd[0]).sum().item(), (vol * Qd[4]).sum().item()
    assert K().cgks_check(ctx) == (0, 0)
    ctx.close()
    for a, b in zip(m0, m1):
        assert abs(b - a) <= 1e-13 * abs(a), (a, b)


def test_walls_in_reduced_precision_track_fp64():
    """BF16x3 reconstruction + FP32 flux with walls against the FP64 GPU path (which matches the
    oracle above): the error level of the periodic precision variants."""
    dims = (20, 18, 16)
    nodes = W.wall_perturbed_nodes(dims)
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    kw = tgv_kw(bc=(2, 2, 1, 1, 2, 2))
    _, Q64, _, _, dts = run_gpu([dims], [nodes], K().default_params(**kw), Q, G, L, 5)
    for rp in (1, 2):
        st, Qr, _, _, _ = run_gpu([dims], [nodes], K().default_params(recon_prec=rp, flux_prec=1, **kw), Q, G, L, 5,
                                  dt=dts[0])
        assert st == (0, 0)
        # the same 5 steps at the first FP64 step size are compared against a fixed-dt FP64 run
        _, Q64f, _, _, _ = run_gpu([dims], [nodes], K().default_params(**kw), Q, G, L, 5, dt=dts[0])
        err = (Qr - Q64f).abs().max().item() / Q64f.abs().max().item()
        assert err < 1e-6, (rp, err)


def test_multiblock_walls_per_block_and_batched_agree_with_oracle():
    dims = [(12, 10, 9), (7, 13, 5)]
    nodes = [W.wall_perturbed_nodes(d) for d in dims]
    states = [W.initial_state(n, W.taylor_green(Ma=0.3), GAM) for n in nodes]
    Q = torch.cat([s[0] for s in states], dim=1)
    G = torch.cat([s[1] for s in states], dim=2)
    L = torch.cat([s[2] for s in states], dim=2)
    kw = tgv_kw(bc=(2, 2, 1, 1, 2, 2))
    dt = 2e-3
    outs = []
    for per_block in (0, 1):
        st, Qd, Gd, Ld, _ = run_gpu(dims, nodes, K().default_params(per_block=per_block, **kw), Q, G, L, 3, dt=dt)
        assert st == (0, 0)
        outs.append((Qd, Gd, Ld))
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)
    off = 0
    for d, n, s in zip(dims, nodes, states):
        N = d[0] * d[1] * d[2]
        ref, sp, _ = PB.oracle_run_pair(d, n, O.params(**kw), *s, 3, dt=dt)
        assert_whole_run(outs[0][0][:, off:off + N], outs[0][1][:, :, off:off + N], outs[0][2][:, :, off:off + N],
                         ref, sp)
        off += N


def test_graph_replay_with_walls_matches_eager():
    dims = (16, 12, 10)
    nodes = mesh("curved_z2", dims)
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    prm = K().default_params(**tgv_kw(bc=(1, 1, 2, 2, 0, 0)))
    st, Qe, Ge, Le, _ = run_gpu([dims], [nodes], prm, Q, G, L, 3)
    ctx = K().Context([dims], [nodes], prm)
    Qd, Gd, Ld = Q.clone().to(dev()), G.clone().to(dev()), L.clone().to(dev())
    dtd = torch.zeros(1, dtype=torch.float64, device=dev())
    for _ in range(3):
        K().cgks_step_graph(ctx, Qd, Gd, Ld, dtd, use_cfl=True)
        torch.cuda.synchronize()
    ctx.close()
    assert torch.equal(Qd, Qe) and torch.equal(Gd, Ge) and torch.equal(Ld, Le)


def _boundary_sample(n, rng, k=40):
    """Cells on every wall side, edge and corner of an n^3 block, plus random interior cells."""
    nx = ny = nz = n
    pick = set()
    for i in (0, nx - 1):
        for j in (0, ny - 1):
            for kk in (0, nz - 1):
                pick.add(i + nx * (j + ny * kk))  # corners
    for _ in range(k):
        c = [int(x) for x in rng.integers(0, n, size=3)]
        c[int(rng.integers(0, 3))] = int(rng.choice([0, n - 1]))  # on a side
        pick.add(c[0] + nx * (c[1] + ny * c[2]))
    pick.update(int(x) for x in rng.choice(n ** 3, size=8, replace=False))
    return np.array(sorted(pick), dtype=np.int64)


@pytest.mark.parametrize("bc", [1, 2])
def test_walls_stage1_sampled_parity_full_size(bc):
    """Stage 1 of the 256^3 wall box (the bench's wall workload and launch configuration) on
    corner, side and interior cells that the oracle evaluates one by one."""
    n = (256, 256, 256)
    print(f"walls full size bc {bc}", flush=True)
    nodes = W.wall_perturbed_nodes(n, device=dev())
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.1), GAM)
    nodes_h = nodes.cpu()
    del nodes
    kw = tgv_kw(Ma=0.1, bc=(bc,) * 6)
    cells = _boundary_sample(256, np.random.default_rng(29))
    dt = 3.5e-4
    Qh, Gh, Lh = Q.cpu().numpy(), G.cpu().numpy(), L.cpu().numpy()
    ref, sp = PB.stage1_cells_pair(n, nodes_h, O.params(**kw), dt, Qh, Gh, Lh, cells)
    del Qh, Gh, Lh
    ctx = K().Context([n], [nodes_h], K().default_params(**kw))
    dtd = torch.full((1,), dt, dtype=torch.float64, device=dev())
    K().cgks_stage(ctx, 1, dtd, Q, G, L)
    torch.cuda.synchronize()
    assert K().cgks_check(ctx) == (0, 0)
    ci = torch.from_numpy(cells).to(dev())
    got = (Q[:, ci].cpu(), G[:, :, ci].cpu(), L[:, :, ci].cpu())
    ctx.close()
    del Q, G, L
    torch.cuda.empty_cache()
    assert_whole_run(*got, ref, sp)


def _pulse3d(rho0=1.0, p0=1.0 / GAM, amp=0.02, u=(0.2, 0.0, 0.0)):
    """Gaussian pressure/density pulse at the centre of [0, pi]^3 in a uniform stream."""
    def f(x, y, z):
        r2 = (x - 1.6) ** 2 + (y - 1.5) ** 2 + (z - 1.55) ** 2
        g = amp * torch.exp(-r2 / 0.3 ** 2)
        return rho0 + g, u[0] + 0.0 * x, u[1] + 0.0 * x, u[2] + 0.0 * x, p0 * (1.0 + GAM * g)
    e = p0 / (GAM - 1.0) + 0.5 * rho0 * sum(c * c for c in u)
    return f, (rho0, rho0 * u[0], rho0 * u[1], rho0 * u[2], e)


@pytest.mark.parametrize("bc", [(3,) * 6, (3, 3, 2, 2, 0, 0)])
def test_far_field_parity_with_oracle(bc):
    dims = (20, 18, 16)
    nodes = W.wall_perturbed_nodes(dims)
    if bc[4] == 0:
        nodes[..., 2] *= 2.0
    f, far = _pulse3d(u=(0.2, 0.0, 0.0))
    Q, G, L = W.initial_state(nodes, f, GAM)
    kw = dict(viscous=1, mu0=2e-3, bc=bc)
    st, Qd, Gd, Ld, dts = run_gpu([dims], [nodes], K().default_params(farfield=far, **kw), Q, G, L, 6)
    assert st == (0, 0)
    ref, sp, dto = PB.oracle_run_pair(dims, nodes, O.params(far=far, **kw), Q, G, L, 6)
    assert dts[-1] == pytest.approx(dto, rel=1e-13)
    assert_whole_run(Qd, Gd, Ld, ref, sp)


def test_far_field_keeps_its_free_stream_on_the_gpu():
    dims = (24, 20, 16)
    nodes = W.wall_perturbed_nodes(dims)
    rho, u, p = 1.2, (0.3, -0.2, 0.1), 0.9
    far = (rho, rho * u[0], rho * u[1], rho * u[2], p / (GAM - 1.0) + 0.5 * rho * sum(c * c for c in u))
    Q, G, L = W.initial_state(nodes, W.uniform(rho=rho, u=u[0], v=u[1], w=u[2], p=p), GAM)
    st, Qd, Gd, Ld, _ = run_gpu([dims], [nodes], K().default_params(viscous=1, mu0=0.01, bc=(3,) * 6, farfield=far),
                                Q, G, L, 10)
    assert st == (0, 0)
    assert (Qd.cpu() - Q).abs().max().item() < 1e-13
    assert Gd.abs().max().item() < 1e-11 and Ld.abs().max().item() < 1e-12


@pytest.mark.parametrize("bc,gather", [((4,) * 6, "staged"), ((4,) * 6, "memory"), ((4, 4, 2, 2, 3, 3), "staged"),
                                       ((4, 4, 1, 1, 0, 0), "memory")])
def test_nonreflecting_parity_with_oracle(bc, gather):
    """Non-reflecting sides (alone, and at corners with no-slip walls, far-field sides and
    symmetry planes), six steps against the oracle; the reconstruction's ghost data through
    LDS-staged bricks and through the memory gather.  The field is the Taylor-Green vortex, whose
    gradients at the sides are of order one, so that a wrong ghost or boundary state shows far
    above rounding (a field uniform to rounding at the sides, as a centred pulse, makes G and L
    there differences of equal values; the device's and the host's pow, which the boundary
    state calls, then differ by more than the two oracle builds do)."""
    dims = (20, 18, 16)
    print(f"non-reflecting case bc {bc} gather {gather}", flush=True)
    nodes = W.wall_perturbed_nodes(dims)
    if bc[4] == 0:
        nodes[..., 2] *= 2.0
    Ma = 0.3
    p0 = 1.0 / (GAM * Ma * Ma)
    far = (1.0, 0.0, 0.0, 0.0, p0 / (GAM - 1.0))
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=Ma), GAM)
    kw = dict(viscous=1, mu0=2e-3, bc=bc)
    ctx = K().Context([dims], [nodes], K().default_params(farfield=far, **kw))
    if gather == "memory":
        K().cgks_set_launch(ctx, 1, 1536, 0, 0)
    Qd, Gd, Ld = Q.clone().to(dev()), G.clone().to(dev()), L.clone().to(dev())
    dtd = torch.zeros(1, dtype=torch.float64, device=dev())
    for _ in range(6):
        K().cgks_step(ctx, Qd, Gd, Ld, dtd, use_cfl=True)
    torch.cuda.synchronize()
    assert K().cgks_check(ctx) == (0, 0)
    ctx.close()
    ref, sp, dto = PB.oracle_run_pair(dims, nodes, O.params(far=far, **kw), Q, G, L, 6)
    assert dtd.item() == pytest.approx(dto, rel=1e-13)
    assert_whole_run(Qd, Gd, Ld, ref, sp)


def test_nonreflecting_free_stream_and_refusals_on_the_gpu():
    dims = (24, 20, 16)
    nodes = W.wall_perturbed_nodes(dims)
    rho, u, p = 1.2, (0.3, -0.2, 0.1), 0.9
    far = (rho, rho * u[0], rho * u[1], rho * u[2], p / (GAM - 1.0) + 0.5 * rho * sum(c * c for c in u))
    Q, G, L = W.initial_state(nodes, W.uniform(rho=rho, u=u[0], v=u[1], w=u[2], p=p), GAM)
    st, Qd, Gd, Ld, _ = run_gpu([dims], [nodes], K().default_params(viscous=1, mu0=0.01, bc=(4,) * 6, farfield=far),
                                Q, G, L, 10)
    assert st == (0, 0)
    assert (Qd.cpu() - Q).abs().max().item() < 1e-13
    assert Gd.abs().max().item() < 1e-11 and Ld.abs().max().item() < 1e-12
    with pytest.raises(RuntimeError):  # learned weights need the same continuation in their inputs
        K().Context([dims], [nodes], K().default_params(weights=1, bc=(4,) * 6, farfield=far))
    with pytest.raises(RuntimeError):  # the outside state must be physical
        K().Context([dims], [nodes], K().default_params(bc=(4,) * 6, farfield=(1.0, 0.0, 0.0, 0.0, -1.0)))
    with pytest.raises(RuntimeError):
        K().Context([dims], [nodes], K().default_params(bc=(5, 5, 0, 0, 0, 0)))


@pytest.mark.parametrize("mode,bc", [("sin", 2), ("cos", 1)])
def test_shear_wave_decays_at_the_viscous_rate_on_the_gpu(mode, bc):
    """A long run of the wall path: the shear wave between no-slip walls (sin profile) or
    symmetry planes (cos profile) decays at exp(-nu pi^2 t / H^2), the closed form the oracle is
    pinned to, over 250 steps at 48 cells across (stretched toward the walls)."""
    H, U, mu0 = 1.0, 0.05, 0.01
    dims = (2, 48, 2)
    nodes = W.stretched_nodes(dims, half=(0.25, H, 0.25), cells_per_half=dims, amp=(0.0, 0.08, 0.0))
    Q, G, L = W.initial_state(nodes, W.shear_wave(U=U, H=H, mode=mode), GAM)
    st, Qd, _, _, dts = run_gpu([dims], [nodes], K().default_params(viscous=1, mu0=mu0, Pr=1.0,
                                                                    bc=(0, 0, bc, bc, 0, 0)), Q, G, L, 250)
    assert st == (0, 0)
    t = sum(dts)
    decay = math.exp(-mu0 * math.pi ** 2 * t / H ** 2)
    assert 1.0 - decay > 0.08, t  # t = 1.01: 9.5 % decay
    rel = (Qd[1].cpu() - decay * Q[1]).abs().max().item() / (U * decay)
    assert rel < 5e-4, rel  # the oracle's own error here: 5e-5 (sin) and 6e-5 (cos)
