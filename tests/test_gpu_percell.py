"""Reconstruction with per-cell stored matrices (recon_impl 2), the comparison baseline for the
shared standard-cell matrix of Sec. 4: whole steps agree with the FP64 oracle and with the
matrix-core path, on single and multi-block meshes whose cell counts are not multiples of the
12-cell storage tiles."""

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2508_08965_amd import workloads as W
import parity_bar as PB
from test_gpu_parity import assert_whole_run

pytestmark = pytest.mark.gpu
GAM = 1.4
TOL = 1e-12


def K():
    from paper_2508_08965_amd import cgks
    return cgks


def dev():
    return torch.device("cuda:0")


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def tgv_kw():
    p0 = 1.0 / (GAM * 0.3 ** 2)
    return dict(viscous=1, visc_law=1, mu0=1.0 / 1600, T_ref=p0, S_suth=p0 * 110.4 / 288.15, Pr=0.72,
                prandtl_fix=1)


def steps(dims, nodes, prm, state, nsteps):
    ctx = K().Context(dims, nodes, prm)
    Q, G, L = (t.clone().to(dev()) for t in state)
    dt = torch.zeros(1, dtype=torch.float64, device=dev())
    for _ in range(nsteps):
        K().cgks_step(ctx, Q, G, L, dt, use_cfl=True)
    torch.cuda.synchronize()
    st = K().cgks_check(ctx)
    ctx.close()
    return st, Q.cpu().numpy(), G.cpu().numpy(), L.cpu().numpy()


def test_percell_steps_match_oracle_curvilinear():
    n = (13, 11, 9)  # 1287 cells: 107 full storage tiles and a ragged one
    nodes = W.perturbed_nodes(n, amp=0.05)
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    st, Qg, Gg, Lg = steps([n], [nodes], K().default_params(recon_impl=2, **tgv_kw()), (Q, G, L), 3)
    assert st == (0, 0)
    ref, sp, _ = PB.oracle_run_pair(n, nodes, O.params(**tgv_kw()), Q, G, L, 3)
    # G and L are built from interface values: the measured bar of the other whole-step tests
    assert_whole_run(Qg, Gg, Lg, ref, sp)


@pytest.mark.parametrize("linear", [0, 1])
def test_percell_matches_matrix_cores_multiblock(linear):
    dims = [(17, 12, 10), (9, 20, 7), (24, 8, 6)]  # block offsets are not multiples of 12
    nodes, states = [], []
    for b, n in enumerate(dims):
        nd = W.perturbed_nodes(n, amp=0.05)
        nodes.append(nd)
        states.append(W.initial_state(nd, W.isotropic_turbulence(16, k0=4.0, Mt=0.5, seed=8965 + b), GAM))
    state = tuple(torch.cat([s[i] for s in states], dim=1 if i == 0 else 2).contiguous() for i in range(3))
    kw = dict(viscous=1, visc_law=0, mu0=2.0e-3, Pr=0.72, prandtl_fix=1, linear=linear)
    a = steps(dims, nodes, K().default_params(recon_impl=2, **kw), state, 2)
    b = steps(dims, nodes, K().default_params(**kw), state, 2)
    assert a[0] == b[0] == (0, 0)
    assert rel(a[1], b[1]) <= TOL
    # each block against the oracle (global CFL step: the minimum over the blocks), G and L
    # within the oracle's measured spread
    prm = O.params(**kw)
    cur = [tuple(t.numpy() for t in s) for s in states]
    alt = [PB.jitter_state(*c) for c in cur]
    for _ in range(2):
        dt = min(O.cfl_dt(n, nd.numpy(), prm, c[0]) for n, nd, c in zip(dims, nodes, cur))
        da = min(O.cfl_dt(n, nd.numpy(), prm, c[0]) for n, nd, c in zip(dims, nodes, alt))
        nxt, nxa = [], []
        for n, nd, c, ca in zip(dims, nodes, cur, alt):
            so, *r = O.run(n, nd.numpy(), prm, *c, 1, dt=dt)[:4]
            sa, *ra = O.run(n, nd.numpy(), prm, *ca, 1, dt=da, variant="fma")[:4]
            assert so == sa == 0
            nxt.append(tuple(r))
            nxa.append(tuple(ra))
        cur, alt = nxt, nxa
    ref = [np.concatenate([c[i] for c in cur], axis=-1) for i in range(3)]
    oth = [np.concatenate([c[i] for c in alt], axis=-1) for i in range(3)]
    sp = {k: PB.spread(x, y) for k, x, y in zip("QGL", ref, oth)}
    for got in (a, b):
        assert_whole_run(*got[1:], ref, sp)
