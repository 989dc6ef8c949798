"""Learned blend weights (the MLP extension of Sec. 3.3) over whole steps, against the oracle
running its own network: no weight computed by the GPU enters the oracle.

Per stage the oracle forms the features and the jump flags of every cell from the stage's
state, evaluates the MLP in FP64 on the BF16-rounded parameters and features, takes GENO's
weights where the jump flag is set, and blends with those weights.  The GPU runs BF16 inference
(FP32 accumulation, hidden activations rounded to BF16): its outputs differ from the FP64
network's by at most sum_j |W2_oj| (2^-8 h_j + 1e-6) + 1e-6 (the bound of
test_bf16_inference_within_its_rounding_bound).  The bar is derived from that bound: a second
oracle run moves every logit by it (random sign) and the GPU must stay within twice the
spread that produces, per variable group of Q, G and L.
"""
import numpy as np
import pytest
import torch

import parity_bar as PB
from oracle import oracle as O
from paper_2508_08965_amd import workloads as W

pytestmark = pytest.mark.gpu

GAM = 1.4
HIT_KW = dict(viscous=1, visc_law=0, mu0=1.44e-3, Pr=0.72, prandtl_fix=1)
NW1, NB1, NW2 = 32 * 18, 32, 7 * 32


def K():
    from paper_2508_08965_amd import cgks
    return cgks


def net_params(seed=11):
    """A network shaped like a trained one: small random weights and a chi logit biased to
    ~5 (chi ~ 0.99 where the features are small, lower where they are not), so that the blend
    is mostly high order, as GENO's is in smooth cells."""
    w = np.random.default_rng(seed).normal(scale=0.15, size=NW1 + NB1 + NW2 + 7).astype(np.float32)
    w[NW1 + NB1 + NW2] = 5.0
    wb = w.astype(np.float64)
    wb[:NW1] = O.bf16(wb[:NW1])                                   # weights in BF16, biases FP32
    wb[NW1 + NB1:NW1 + NB1 + NW2] = O.bf16(wb[NW1 + NB1:NW1 + NB1 + NW2])
    return w, wb


def outputs(wb, H, shift=None):
    """chi (sigmoid) and omega (softmax) from the hidden activations, logits optionally moved."""
    W2 = wb[NW1 + NB1:NW1 + NB1 + NW2].reshape(7, 32)
    b2 = wb[NW1 + NB1 + NW2:]
    z = H @ W2.T + b2
    if shift is not None:
        z = z + shift
    y = np.empty_like(z)
    y[:, 0] = 1.0 / (1.0 + np.exp(-z[:, 0]))
    e = np.exp(z[:, 1:] - z[:, 1:].max(axis=1, keepdims=True))
    y[:, 1:] = e / e.sum(axis=1, keepdims=True)
    return y


def oracle_learned_run(n, nodes, prm, wb, state, steps, seed=None, stats=None):
    N = n[0] * n[1] * n[2]
    cells = np.arange(N)
    q, g, l = (np.array(a.numpy() if hasattr(a, "numpy") else a, dtype=np.float64) for a in state)
    stash = np.zeros((90, N))
    rng = np.random.default_rng(seed) if seed is not None else None
    W2abs = np.abs(wb[NW1 + NB1:NW1 + NB1 + NW2].reshape(7, 32))
    for _ in range(steps):
        dt = O.cfl_dt(n, nodes, prm, q)
        for s in (1, 2):
            X, jump = O.features(n, nodes, prm, q, l, cells, thresh=0.05)
            Y, H = O.mlp_forward(wb, O.bf16(X.reshape(-1, 18)))
            if rng is not None:
                bound = (2.0 ** -8 * H + 1e-6) @ W2abs.T + 1e-6
                Y = outputs(wb, H, shift=bound * rng.choice([-1.0, 1.0], size=bound.shape))
            _, wg = O.recon_weights(n, nodes, prm, q, g, l, cells)
            win = np.where(jump[:, None, None], wg, Y.reshape(N, 5, 7))
            if stats is not None:
                stats.append((float(jump.mean()), float((win[:, :, 0] < 0.99).mean())))
            assert O.stage_weights(n, nodes, prm, s, dt, q, g, l, stash, win) == 0
    return q, g, l


def test_learned_steps_match_the_oracles_own_network():
    n = (16, 14, 12)
    nodes = W.perturbed_nodes(n, amp=0.05)
    Q, G, L = W.initial_state(nodes, W.isotropic_turbulence(32, k0=8.0, Mt=1.0, seed=8967), GAM)
    w32, wb = net_params()
    steps = 3
    # GPU: learned weights with GENO where the jump indicator fires
    ctx = K().Context([n], [nodes], K().default_params(weights=1, **HIT_KW))
    K().cgks_mlp_set(ctx, w32)
    Qd, Gd, Ld = Q.to("cuda:0"), G.to("cuda:0"), L.to("cuda:0")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    for _ in range(steps):
        K().cgks_step(ctx, Qd, Gd, Ld, dt, use_cfl=True)
    torch.cuda.synchronize()
    assert K().cgks_check(ctx) == (0, 0)
    ctx.close()
    prm = O.params(**HIT_KW)
    stats = []
    ref = oracle_learned_run(n, nodes.numpy(), prm, wb, (Q, G, L), steps, stats=stats)
    alt = oracle_learned_run(n, nodes.numpy(), prm, wb, (Q, G, L), steps, seed=5)
    # both branches are exercised: some cells take GENO (jump), most take the network
    jf = np.mean([a for a, _ in stats])
    assert 0.01 < jf < 0.9, jf
    assert min(b for _, b in stats) > 0.001
    for kind, gpu, r, a in zip("QGL", (Qd, Gd, Ld), ref, alt):
        sp = PB.spread(r, a)
        assert all(sp[grp]["diff"] > 0 for grp in PB.GROUPS)
        PB.assert_spread_parity(gpu, r, sp, kind)
