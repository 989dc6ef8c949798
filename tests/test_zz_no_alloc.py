"""cgks_dt_noalloc, the time step for callers that cannot allocate, against cgks_dt through the
C ABI: the same step (bitwise: both take the minimum over the same partition) on two calls in a
row, the second on a smaller mesh than the first, then the first mesh again."""
import math

import pytest
import torch

from paper_2508_08965_amd import workloads as W

pytestmark = pytest.mark.gpu

GAM = 1.4


def K():
    from paper_2508_08965_amd import cgks
    return cgks


def case(n, viscous):
    nodes = W.perturbed_nodes(n, amp=0.05)
    Q, _, _ = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    kw = dict(viscous=1, visc_law=1, mu0=0.05, T_ref=1.0 / (GAM * 0.09), S_suth=0.3, Pr=0.72,
              prandtl_fix=1) if viscous else {}
    ctx = K().Context([n], [nodes], K().default_params(**kw))
    return ctx, Q.to("cuda:0")


def both(ctx, Q):
    a = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    b = torch.full((1,), -2.0, dtype=torch.float64, device="cuda:0")
    K().cgks_dt(ctx, Q, a)
    K().cgks_dt_noalloc(ctx, Q, b)
    torch.cuda.synchronize()
    assert K().cgks_check(ctx) == (0, 0)
    return a.item(), b.item()


@pytest.mark.parametrize("viscous", [0, 1])
def test_noalloc_dt_equals_dt_on_consecutive_calls(viscous):
    big = case((48, 40, 36), viscous)     # 69,120 cells: 270 partial minima
    small = case((9, 7, 5), viscous)      # 315 cells: 2 partial minima
    try:
        for ctx, Q in (big, small, big):
            ref, got = both(ctx, Q)
            assert math.isfinite(ref) and ref > 0
            assert got == ref
    finally:
        big[0].close()
        small[0].close()


def test_noalloc_dt_rejects_null_arguments():
    ctx, Q = case((4, 4, 4), 0)
    try:
        dt = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        assert K().lib().cgks_dt_noalloc(ctx.h, None, dt.data_ptr(), None) == K().EINVAL
        assert K().lib().cgks_dt_noalloc(ctx.h, Q.data_ptr(), None, None) == K().EINVAL
        assert K().lib().cgks_dt_noalloc(None, Q.data_ptr(), dt.data_ptr(), None) == K().EINVAL
    finally:
        ctx.close()
