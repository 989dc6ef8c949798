"""The reconstruction with bricks staged in LDS (cgks_launch.stage = 1).

It gathers the same neighbour data as the reconstruction that reads memory and runs the same
arithmetic, but it is another instantiation of the kernel, and the compiler may fuse its
multiply-adds differently: results agree to rounding, not bitwise.  So the staged path is held
to the FP64 parity bar against the oracle itself (ragged bricks of three shapes on the
curvilinear mesh, walls and far-field sides), and against the memory-gathering path within
the oracle's own rounding spread (uneven multi-block meshes with blocks one cell thick, learned
weights) or at the FP32x3 level for that reconstruction.  Invalid staged configurations are
refused."""
import numpy as np
import pytest
import torch

import parity_bar as PB
from oracle import oracle as O
from paper_2508_08965_amd import workloads as W

pytestmark = pytest.mark.gpu

GAM = 1.4


def K():
    from paper_2508_08965_amd import cgks
    return cgks


def tgv_kw(Ma=0.3, **extra):
    p0 = 1.0 / (GAM * Ma * Ma)
    kw = dict(viscous=1, visc_law=1, mu0=1.0 / 1600.0, T_ref=p0, S_suth=p0 * 110.4 / 288.15, Pr=0.72,
              prandtl_fix=1)
    kw.update(extra)
    return kw


def run(dims, nodes, states, prm, steps, stage=None, setup=None, dt_fixed=None):
    ctx = K().Context(dims, nodes, prm)
    if setup:
        setup(ctx)
    if stage:
        K().cgks_set_launch(ctx, 1, 16, 0, 0, brick_y=stage[0], brick_z=stage[1], stage=1)
        assert K().cgks_get_launch(ctx, 1)["stage"] == 1
    Q = torch.cat([s[0] for s in states], dim=1).contiguous().to("cuda:0")
    G = torch.cat([s[1] for s in states], dim=2).contiguous().to("cuda:0")
    L = torch.cat([s[2] for s in states], dim=2).contiguous().to("cuda:0")
    dt = torch.full((1,), dt_fixed or 0.0, dtype=torch.float64, device="cuda:0")
    for _ in range(steps):
        K().cgks_step(ctx, Q, G, L, dt, use_cfl=dt_fixed is None)
    torch.cuda.synchronize()
    st = K().cgks_check(ctx)
    ctx.close()
    assert st == (0, 0)
    return Q, G, L


def against(got, ref, sp):
    PB.assert_rel(got[0], ref[0], "Q")
    PB.assert_spread_parity(got[1], ref[1], sp["G"], "G")
    PB.assert_spread_parity(got[2], ref[2], sp["L"], "L")


@pytest.mark.parametrize("brick", [(10, 8), (4, 3), (1, 1)])
def test_staged_matches_oracle_curvilinear(brick):
    n = (37, 23, 19)  # ragged in every direction for every brick
    nodes = W.perturbed_nodes(n, amp=0.05)
    st = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    ref, sp, _ = PB.oracle_run_pair(n, nodes, O.params(**tgv_kw()), *st, 3)
    against(run([n], [nodes], [st], K().default_params(**tgv_kw()), 3, stage=brick), ref, sp)


@pytest.mark.parametrize("bc", [(1,) * 6, (2,) * 6, (1, 1, 2, 2, 0, 0), (3,) * 6])
def test_staged_matches_oracle_with_walls(bc):
    n = (20, 18, 16)
    nodes = W.wall_perturbed_nodes(n)
    if bc[4] == 0:
        nodes[..., 2] *= 2.0
    st = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    far = (1.0, 0.1, 0.0, 0.0, 1.0 / (GAM * 0.09 * (GAM - 1.0)) + 0.005)
    ref, sp, _ = PB.oracle_run_pair(n, nodes, O.params(far=far, **tgv_kw(bc=bc)), *st, 3)
    got = run([n], [nodes], [st], K().default_params(**tgv_kw(bc=bc, farfield=far)), 3, stage=(6, 5))
    against(got, ref, sp)


def oracle_spread_blocks(dims, nodes, states, prm, steps, dt):
    """The oracle's rounding spread of a multi-block run at a fixed step (blocks independent)."""
    refs, alts = [], []
    for n, nd, s in zip(dims, nodes, states):
        ref, _, _ = PB.oracle_run_pair(n, nd, prm, *s, steps, dt=dt)
        st, *alt = O.run(n, nd.numpy(), prm, *PB.jitter_state(*s), steps, dt=dt, variant="fma")[:4]
        assert st == 0
        refs.append(ref)
        alts.append(alt)
    cat = lambda xs, i: np.concatenate([x[i] for x in xs], axis=-1)
    return {k: PB.spread(cat(refs, i), cat(alts, i)) for i, k in enumerate("QGL")}


def test_staged_matches_memory_gather_multiblock_and_thin_blocks():
    dims = [(40, 12, 9), (7, 33, 5), (1, 9, 6), (13, 1, 4), (5, 6, 1), (17, 17, 17)]
    nodes = [W.perturbed_nodes(d, amp=0.05 if min(d) > 1 else 0.0) for d in dims]
    st = [W.initial_state(nd, W.isotropic_turbulence(16, k0=4.0, Mt=0.5, seed=9100 + b), GAM)
          for b, nd in enumerate(nodes)]
    T0 = 1.0 / GAM
    kw = dict(viscous=1, visc_law=1, mu0=2e-3, T_ref=T0, S_suth=T0 * 110.4 / 288.15, Pr=0.72, prandtl_fix=1)
    dt = 2e-3
    sp = oracle_spread_blocks(dims, nodes, st, O.params(**kw), 2, dt)
    ref = run(dims, nodes, st, K().default_params(**kw), 2, dt_fixed=dt)
    got = run(dims, nodes, st, K().default_params(**kw), 2, stage=(10, 8), dt_fixed=dt)
    for kind, a, b in zip("QGL", got, ref):
        PB.assert_spread_parity(a, b, sp[kind], kind)


def test_staged_learned_weights_and_fp32x3():
    n = (24, 20, 18)
    nodes = W.perturbed_nodes(n, amp=0.05)
    st = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    # FP32x3 contractions: the staged and memory-gathering forms agree at the FP32 level
    prm = K().default_params(recon_prec=1, flux_prec=1, **tgv_kw())
    a, b = run([n], [nodes], [st], prm, 2), run([n], [nodes], [st], prm, 2, stage=(10, 8))
    for x, y in zip(a, b):
        PB.assert_rel(x, y, "fp32x3", tol=1e-6)
    # learned weights (FP64 reconstruction): within the oracle's spread of the GENO run
    _, sp, _ = PB.oracle_run_pair(n, nodes, O.params(**tgv_kw()), *st, 2)
    prm = K().default_params(weights=1, **tgv_kw())
    setup = lambda c: K().cgks_mlp_init(c, 7)
    a = run([n], [nodes], [st], prm, 2, setup=setup)
    b = run([n], [nodes], [st], prm, 2, stage=(10, 8), setup=setup)
    PB.assert_rel(b[0], a[0], "Q")
    PB.assert_spread_parity(b[1], a[1], sp["G"], "G")
    PB.assert_spread_parity(b[2], a[2], sp["L"], "L")


def test_invalid_staged_configurations_refused():
    n = (8, 8, 8)
    nodes = W.cartesian_nodes(n)
    ctx = K().Context([n], [nodes], K().default_params())
    for cfg in [dict(tile_cells=32, brick_y=4, brick_z=4), dict(tile_cells=16, brick_y=0, brick_z=0),
                dict(tile_cells=16, brick_y=12, brick_z=9)]:
        with pytest.raises(RuntimeError):
            K().cgks_set_launch(ctx, 1, cfg["tile_cells"], 0, 0, brick_y=cfg["brick_y"], brick_z=cfg["brick_z"],
                                stage=1)
    ctx.close()
    ctx = K().Context([n], [nodes], K().default_params(recon_prec=2, flux_prec=1))
    with pytest.raises(RuntimeError):
        K().cgks_set_launch(ctx, 1, 16, 0, 0, brick_y=4, brick_z=4, stage=1)
    ctx.close()
