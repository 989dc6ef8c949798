"""The Gauss-point buffer with padded rows on the GPU, against the oracle.

The buffer pads a block's rows to a multiple of 16 cells where that costs at most a quarter
more: x extents 53 and 65 are padded (to 64 and 80), 17 is not.  These blocks go through every
reconstruction form (matrix cores staged and gathered from memory, vector ALU, per-cell stored
matrices, the FP32x3 and BF16x3 splits), the flux, the wall-face flux and the export of the
Gauss-point values, each of which indexes the buffer through the padded layout; a wrong index
shows at the size of the data, far above the bars used here."""
import numpy as np
import pytest
import torch

import parity_bar as PB
from oracle import oracle as O
from paper_2508_08965_amd import workloads as W

pytestmark = pytest.mark.gpu
GAM = 1.4
TOL = 1e-12
DIMS = [(53, 6, 5), (65, 4, 3), (17, 5, 4)]


def K():
    from paper_2508_08965_amd import cgks
    return cgks


def dev():
    return torch.device("cuda:0")


def hit_kw():
    return dict(viscous=1, visc_law=0, mu0=2.0e-3, Pr=0.72, prandtl_fix=1)


@pytest.mark.parametrize("impl,prec,tol", [(0, 0, TOL), (1, 0, TOL), (2, 0, TOL), (0, 1, 1e-5), (0, 2, 1e-4)])
def test_padded_reconstruction_export_matches_oracle(impl, prec, tol):
    n = DIMS[0]
    print(f"padded reconstruction impl {impl} prec {prec}", flush=True)
    nodes = W.perturbed_nodes(n, amp=0.05)
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    ref = O.recon(n, nodes.numpy(), O.params(), Q.numpy(), G.numpy(), L.numpy(), np.arange(Q.shape[1]))
    ctx = K().Context([n], [nodes], K().default_params(recon_impl=impl, recon_prec=prec))
    gp = torch.zeros(Q.shape[1], 24, 5, 4, dtype=torch.float64, device=dev())
    K().cgks_recon(ctx, Q.to(dev()), G.to(dev()), L.to(dev()), gp)
    torch.cuda.synchronize()
    ctx.close()
    out = gp.cpu().numpy()
    for v in range(5):
        for c in range(4):
            scale = max(np.abs(ref[:, :, v, c]).max(), 1e-300)
            assert np.abs(out[:, :, v, c] - ref[:, :, v, c]).max() <= tol * scale, (v, c)


@pytest.mark.parametrize("gather", ["staged", "memory"])
def test_padded_multiblock_steps_match_oracle(gather):
    nodes, states = [], []
    for b, n in enumerate(DIMS):
        nd = W.perturbed_nodes(n, amp=0.05)
        nodes.append(nd)
        states.append(W.initial_state(nd, W.isotropic_turbulence(16, k0=4.0, Mt=0.5, seed=8965 + b), GAM))
    kw = hit_kw()
    ctx = K().Context(DIMS, nodes, K().default_params(**kw))
    if gather == "memory":
        K().cgks_set_launch(ctx, 1, 1536, 0, 0)
    Q, G, L = (torch.cat([s[i] for s in states], dim=-1).contiguous().to(dev()) for i in range(3))
    dt = torch.zeros(1, dtype=torch.float64, device=dev())
    dts = []
    for _ in range(2):
        K().cgks_step(ctx, Q, G, L, dt, use_cfl=True)
        dts.append(dt.item())
    torch.cuda.synchronize()
    assert K().cgks_check(ctx) == (0, 0)
    ctx.close()
    cur = [tuple(t.numpy().copy() for t in s) for s in states]
    for step in range(2):
        dto = min(O.cfl_dt(n, nd.numpy(), O.params(**kw), c[0]) for n, nd, c in zip(DIMS, nodes, cur))
        assert abs(dto - dts[step]) <= 1e-13 * dto
        nxt = []
        for n, nd, c in zip(DIMS, nodes, cur):
            so, Qo, Go, Lo, _, _ = O.run(n, nd.numpy(), O.params(**kw), c[0], c[1], c[2], 1, dt=dto)
            assert so == 0
            nxt.append((Qo, Go, Lo))
        cur = nxt
    for i, g in enumerate((Q, G, L)):
        ref = np.concatenate([c[i] for c in cur], axis=-1)
        assert np.linalg.norm(g.cpu().numpy() - ref) <= TOL * np.linalg.norm(ref), i


def test_padded_walls_steps_match_oracle():
    """Symmetry planes in x, no-slip walls in y, periodic z on a padded block: the wall-face
    flux reads the padded records of both walls of a line."""
    n = DIMS[0]
    nodes = W.wall_perturbed_nodes(n)
    nodes[..., 2] *= 2.0
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    p0 = 1.0 / (GAM * 0.09)
    kw = dict(viscous=1, visc_law=1, mu0=1.0 / 1600, T_ref=p0, S_suth=p0 * 110.4 / 288.15, Pr=0.72,
              prandtl_fix=1, bc=(1, 1, 2, 2, 0, 0))
    ctx = K().Context([n], [nodes], K().default_params(**kw))
    Qd, Gd, Ld = Q.clone().to(dev()), G.clone().to(dev()), L.clone().to(dev())
    dt = torch.zeros(1, dtype=torch.float64, device=dev())
    for _ in range(3):
        K().cgks_step(ctx, Qd, Gd, Ld, dt, use_cfl=True)
    torch.cuda.synchronize()
    assert K().cgks_check(ctx) == (0, 0)
    ctx.close()
    (Qo, Go, Lo), sp, dto = PB.oracle_run_pair(n, nodes, O.params(**kw), Q, G, L, 3)
    assert dt.item() == pytest.approx(dto, rel=1e-13)
    PB.assert_rel(Qd, Qo, "Q")
    PB.assert_spread_parity(Gd, Go, sp["G"], "G")
    PB.assert_spread_parity(Ld, Lo, sp["L"], "L")
