"""The Python binding refuses arrays that are too small for the context before any launch, so a
wrong shape never reaches a kernel."""
import pytest
import torch

from paper_2508_08965_amd import workloads as W

pytestmark = pytest.mark.gpu


def K():
    from paper_2508_08965_amd import cgks
    return cgks


def test_undersized_arrays_are_rejected_on_the_host():
    n = (6, 5, 4)
    N = 6 * 5 * 4
    ctx = K().Context([n], [W.cartesian_nodes(n)], K().default_params())
    dev = torch.device("cuda:0")
    Q = torch.ones(5, N, dtype=torch.float64, device=dev)
    G = torch.zeros(5, 3, N, dtype=torch.float64, device=dev)
    L = torch.zeros(5, 12, N, dtype=torch.float64, device=dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    small = torch.zeros(5, N - 1, dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):
        K().cgks_step(ctx, small, G, L, dt)
    with pytest.raises(ValueError):
        K().cgks_step(ctx, Q, G[:, :2].contiguous(), L, dt)
    with pytest.raises(ValueError):
        K().cgks_stage(ctx, 1, dt, Q, G, L[:, :11].contiguous())
    with pytest.raises(ValueError):
        K().cgks_recon(ctx, Q, G, L, torch.zeros(N, 24, 5, 3, dtype=torch.float64, device=dev))
    with pytest.raises(ValueError):
        K().cgks_step(ctx, Q.float(), G, L, dt)  # wrong dtype
    with pytest.raises(ValueError):
        K().cgks_dt(ctx, Q, torch.zeros(0, dtype=torch.float64, device=dev))
    # the correct shapes still run
    Q[4] = 2.5
    K().cgks_dt(ctx, Q, dt)
    torch.cuda.synchronize()
    assert dt.item() > 0
    ctx.close()
