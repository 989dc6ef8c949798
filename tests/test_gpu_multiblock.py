"""Multi-block batching on the GPU: one launch per kernel over a work list spanning uneven
periodic blocks, per-block launches, launch configurations, the autotuner and graph replay.

Every block is an independent periodic box, so the FP64 oracle advances each block on its
own; the CFL step of the multi-block mesh is the minimum over all cells of all blocks, i.e.
the minimum of the blocks' own CFL steps.  The arithmetic of a cell does not depend on how
the cells are split into tiles or launches, so all launch variants must agree bitwise."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2508_08965_amd import workloads as W

pytestmark = pytest.mark.gpu
GAM = 1.4
TOL = 1e-12

# uneven blocks with ragged tails for every tile size used below
DIMS = [(17, 12, 10), (9, 20, 7), (24, 8, 6)]


def K():
    from paper_2508_08965_amd import cgks
    return cgks


def dev():
    return torch.device("cuda:0")


def hit_kw():
    # decaying isotropic turbulence: rho 1, p 1/gamma, viscous with constant mu
    return dict(viscous=1, visc_law=0, mu0=2.0e-3, Pr=0.72, prandtl_fix=1)


def blocks_state(seed0=8965):
    nodes, states = [], []
    for b, n in enumerate(DIMS):
        nd = W.perturbed_nodes(n, amp=0.05)
        Q, G, L = W.initial_state(nd, W.isotropic_turbulence(16, k0=4.0, Mt=0.5, seed=seed0 + b), GAM)
        nodes.append(nd)
        states.append((Q, G, L))
    return nodes, states


def concat(states):
    Q = torch.cat([s[0] for s in states], dim=1).contiguous()
    G = torch.cat([s[1] for s in states], dim=2).contiguous()
    L = torch.cat([s[2] for s in states], dim=2).contiguous()
    return Q, G, L


def run_gpu(prm, nodes, states, nsteps, configure=None, graph=False):
    ctx = K().Context(DIMS, nodes, prm)
    if configure:
        configure(ctx)
    Q, G, L = (t.to(dev()) for t in concat(states))
    dt = torch.zeros(1, dtype=torch.float64, device=dev())
    dts = []
    for _ in range(nsteps):
        if graph:
            K().cgks_step_graph(ctx, Q, G, L, dt, use_cfl=True)
        else:
            K().cgks_step(ctx, Q, G, L, dt, use_cfl=True)
        dts.append(dt.item())
    torch.cuda.synchronize()
    st = K().cgks_check(ctx)
    ctx.close()
    return st, Q.cpu(), G.cpu(), L.cpu(), dts


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_batched_multiblock_parity_with_oracle():
    nodes, states = blocks_state()
    kw = hit_kw()
    st, Qg, Gg, Lg, dts = run_gpu(K().default_params(**kw), nodes, states, 2)
    assert st == (0, 0)
    # oracle: each block on its own, global CFL step = min over blocks
    cur = [tuple(t.numpy().copy() for t in s) for s in states]
    for step in range(2):
        dt = min(O.cfl_dt(n, nd.numpy(), O.params(**kw), c[0]) for n, nd, c in zip(DIMS, nodes, cur))
        assert abs(dt - dts[step]) <= 1e-13 * dt
        nxt = []
        for n, nd, c in zip(DIMS, nodes, cur):
            so, Qo, Go, Lo, _, _ = O.run(n, nd.numpy(), O.params(**kw), c[0], c[1], c[2], 1, dt=dt)
            assert so == 0
            nxt.append((Qo, Go, Lo))
        cur = nxt
    Qo = np.concatenate([c[0] for c in cur], axis=1)
    Go = np.concatenate([c[1] for c in cur], axis=2)
    Lo = np.concatenate([c[2] for c in cur], axis=2)
    assert rel(Qg.numpy(), Qo) <= TOL
    assert rel(Gg.numpy(), Go) <= TOL
    assert rel(Lg.numpy(), Lo) <= TOL


def test_batched_equals_per_block_launches_bitwise():
    nodes, states = blocks_state()
    a = run_gpu(K().default_params(**hit_kw()), nodes, states, 2)
    b = run_gpu(K().default_params(per_block=1, **hit_kw()), nodes, states, 2)
    assert a[0] == b[0] == (0, 0)
    for x, y in zip(a[1:4], b[1:4]):
        assert torch.equal(x, y)
    assert a[4] == b[4]


def memory_gather(ctx):
    """The reconstruction form that gathers neighbours from memory (runs of 1536 cells): the
    configurations below are compared with it, bitwise (the staged form is another kernel
    instantiation, compared in tests/test_gpu_staged.py)."""
    K().cgks_set_launch(ctx, 1, 1536, 0, 0)


@pytest.mark.parametrize("rtile,rgroups,rxcd,fgroups,fxcd,ugroups,by,bz", [
    (16, 0, 0, 0, 0, 0, 0, 0),
    (48, 8, 1, 0, 1, 8, 0, 0),
    (4096, 3, 0, 0, 0, 1, 0, 0),
    (128, 512, 1, 0, 1, 0, 0, 0),
    (16, 0, 0, 0, 0, 0, 8, 16),   # bricks with ragged edges in x, y and z
    (32, 24, 1, 0, 1, 0, 3, 5),
    (4096, 0, 1, 0, 0, 0, 4096, 4096),  # one brick per block
])
def test_launch_configurations_bitwise(rtile, rgroups, rxcd, fgroups, fxcd, ugroups, by, bz):
    nodes, states = blocks_state()
    ref = run_gpu(K().default_params(**hit_kw()), nodes, states, 2, configure=memory_gather)

    def configure(ctx):
        K().cgks_set_launch(ctx, 1, rtile, rgroups, rxcd, by, bz)
        K().cgks_set_launch(ctx, 2, 128, fgroups, fxcd)
        K().cgks_set_launch(ctx, 3, 256, ugroups, 0)
        assert K().cgks_get_launch(ctx, 1) == {"tile_cells": rtile, "ngroups": rgroups, "xcd": rxcd,
                                              "brick_y": by, "brick_z": bz, "stage": 0}

    got = run_gpu(K().default_params(**hit_kw()), nodes, states, 2, configure=configure)
    assert got[0] == (0, 0)
    for x, y in zip(got[1:4], ref[1:4]):
        assert torch.equal(x, y)


def test_invalid_launch_configurations_rejected():
    nodes, states = blocks_state()
    ctx = K().Context(DIMS, nodes, K().default_params(**hit_kw()))
    for kind, t, g, x, by, bz in [(1, 24, 0, 0, 0, 0), (1, 8192, 0, 0, 0, 0), (2, 64, 0, 0, 0, 0),
                                  (3, 128, 0, 0, 0, 0), (1, 128, 12, 1, 0, 0), (4, 128, 0, 0, 0, 0),
                                  (1, 128, -1, 0, 0, 0), (2, 128, 16, 0, 0, 0), (1, 16, 0, 0, 4, 0),
                                  (1, 16, 0, 0, -1, 2), (3, 256, 0, 0, 2, 2)]:
        with pytest.raises(RuntimeError):
            K().cgks_set_launch(ctx, kind, t, g, x, by, bz)
    ctx.close()


def test_autotune_keeps_results_bitwise():
    nodes, states = blocks_state()
    rep = {}

    def configure(ctx):
        Q, G, L = (t.to(dev()) for t in concat(states))
        dt = torch.full((1,), 1e-3, dtype=torch.float64, device=dev())
        rep["r"] = K().cgks_autotune(ctx, Q, G, L, dt, reps=2)
        rep["stage"] = K().cgks_get_launch(ctx, 1)["stage"]
        # the tuner only reads the state
        for x, y in zip((Q, G, L), concat(states)):
            assert torch.equal(x.cpu(), y)

    got = run_gpu(K().default_params(**hit_kw()), nodes, states, 2, configure=configure)
    assert got[0] == (0, 0)
    # against the default of the form the tuner picked (staged bricks, or memory gather)
    ref = run_gpu(K().default_params(**hit_kw()), nodes, states, 2,
                  configure=None if rep["stage"] else memory_gather)
    kinds = {r["kind"] for r in rep["r"]}
    assert kinds == {"reconstruction", "flux"}
    assert all(r["ms"] > 0 and math.isfinite(r["ms"]) for r in rep["r"])
    for x, y in zip(got[1:4], ref[1:4]):
        assert torch.equal(x, y)


def test_graph_replay_matches_eager_every_replay():
    """Graph replays interleaved with eager work and host synchronisation; each replay is
    checked against the eager path advanced by the same number of steps."""
    nodes, states = blocks_state()
    prm = K().default_params(**hit_kw())
    ctx_e = K().Context(DIMS, nodes, prm)
    ctx_g = K().Context(DIMS, nodes, prm)
    Qe, Ge, Le = (t.to(dev()) for t in concat(states))
    Qg, Gg, Lg = (t.clone() for t in (Qe, Ge, Le))
    dte = torch.zeros(1, dtype=torch.float64, device=dev())
    dtg = torch.zeros(1, dtype=torch.float64, device=dev())
    for rep in range(4):
        K().cgks_step(ctx_e, Qe, Ge, Le, dte, use_cfl=True)
        K().cgks_step_graph(ctx_g, Qg, Gg, Lg, dtg, use_cfl=True)
        scratch = (Qe * 2.0).sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert math.isfinite(float(scratch))
        assert torch.equal(dte, dtg), rep
        for x, y in zip((Qe, Ge, Le), (Qg, Gg, Lg)):
            assert torch.equal(x, y), rep
    assert K().cgks_check(ctx_e) == (0, 0) and K().cgks_check(ctx_g) == (0, 0)
    # new pointers: the context captures a new graph
    Q2, G2, L2 = Qg.clone(), Gg.clone(), Lg.clone()
    K().cgks_step_graph(ctx_g, Q2, G2, L2, dtg, use_cfl=True)
    K().cgks_step(ctx_e, Qe, Ge, Le, dte, use_cfl=True)
    torch.cuda.synchronize()
    for x, y in zip((Qe, Ge, Le), (Q2, G2, L2)):
        assert torch.equal(x, y)
    ctx_e.close()
    ctx_g.close()


@pytest.mark.parametrize("recon_prec,flux_prec", [(1, 1), (2, 1), (2, 0)])
def test_reduced_precision_batched_equals_per_block_and_bricks(recon_prec, flux_prec):
    """The split-precision kernels also take their work from the tile list: batched, per-block
    and brick launches agree bitwise, and stay close to the FP64 path."""
    nodes, states = blocks_state()
    kw = dict(recon_prec=recon_prec, flux_prec=flux_prec, **hit_kw())
    # the memory-gathering form throughout (the staged FP32x3 form: tests/test_gpu_staged.py)
    a = run_gpu(K().default_params(**kw), nodes, states, 2, configure=memory_gather)
    b = run_gpu(K().default_params(per_block=1, **kw), nodes, states, 2, configure=memory_gather)
    c = run_gpu(K().default_params(**kw), nodes, states, 2,
                configure=lambda ctx: K().cgks_set_launch(ctx, 1, 32, 0, 1, 3, 5))
    ref = run_gpu(K().default_params(**hit_kw()), nodes, states, 2)
    assert a[0] == b[0] == c[0] == (0, 0)
    for x, y, z in zip(a[1:4], b[1:4], c[1:4]):
        assert torch.equal(x, y) and torch.equal(x, z)
    assert rel(a[1].numpy(), ref[1].numpy()) <= 1e-5


def test_degenerate_blocks_one_cell_thick_parity_with_oracle():
    """Blocks one cell thick along x, y or z (periodic: the cell is its own neighbour there), in
    one multi-block mesh: each block follows the oracle."""
    dims = [(1, 9, 6), (13, 1, 4), (5, 6, 1)]
    nodes, states = [], []
    for b, n in enumerate(dims):
        nd = W.perturbed_nodes(n, amp=0.0)  # Cartesian: a one-cell axis keeps a flat metric
        nodes.append(nd)
        states.append(W.initial_state(nd, W.isotropic_turbulence(16, k0=4.0, Mt=0.3, seed=9000 + b), GAM))
    kw = hit_kw()
    ctx = K().Context(dims, nodes, K().default_params(**kw))
    Q, G, L = (t.to(dev()) for t in concat(states))
    dt = torch.full((1,), 1e-3, dtype=torch.float64, device=dev())
    K().cgks_step(ctx, Q, G, L, dt, use_cfl=False)
    torch.cuda.synchronize()
    assert K().cgks_check(ctx) == (0, 0)
    ctx.close()
    off = 0
    for n, nd, s in zip(dims, nodes, states):
        N = n[0] * n[1] * n[2]
        so, Qo, Go, Lo, _, _ = O.run(n, nd.numpy(), O.params(**kw), s[0].numpy(), s[1].numpy(), s[2].numpy(), 1,
                                     dt=1e-3)
        assert so == 0
        assert rel(Q[:, off:off + N].cpu().numpy(), Qo) <= TOL, n
        off += N
