"""Reduced-precision variants of the HIP path (FP32x3 or BF16x3 split-precision reconstruction
on the FP32 or BF16 matrix cores, FP32 gas-kinetic flux; metrics and S2O4 accumulation FP64)
against the FP64 oracle.  These are accuracy reports with bounds derived from FP32 rounding, not parity
at 1e-12: the FP32 flux evaluates values of size ~p (71 at Ma 0.1) whose face-to-face
differences are ~1e-2 of that, so single-precision rounding (6e-8) leaves ~1e-5 relative
error in a flux divergence; after a few steps the state differs from FP64 by ~1e-6."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2508_08965_amd import workloads as W

pytestmark = pytest.mark.gpu
GAM = 1.4


def K():
    from paper_2508_08965_amd import cgks
    return cgks


def dev():
    return torch.device("cuda:0")


def cons(rho, u, p):
    return np.array([rho, rho * u[0], rho * u[1], rho * u[2], p / (GAM - 1) + 0.5 * rho * np.dot(u, u)])


def test_fp32_flux_points_accuracy():
    rng = np.random.default_rng(41)
    npts = 515
    ql = np.array([cons(rng.uniform(0.5, 2), rng.uniform(-1, 1, 3), rng.uniform(0.5, 2)) for _ in range(npts)])
    qr = np.array([cons(rng.uniform(0.5, 2), rng.uniform(-1, 1, 3), rng.uniform(0.5, 2)) for _ in range(npts)])
    gl = rng.normal(scale=0.5, size=(npts, 5, 3))
    gr = rng.normal(scale=0.5, size=(npts, 5, 3))
    nrm = rng.normal(size=(npts, 3))
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    kw = dict(viscous=1, visc_law=1, mu0=0.01, T_ref=1.0, S_suth=0.38, Pr=0.72, prandtl_fix=1)
    st, F, Ft, S = O.flux(O.params(**kw), ql, gl, qr, gr, nrm, 0.013)
    assert st == 0
    ctx = K().Context([(2, 2, 2)], [W.cartesian_nodes((2, 2, 2))], K().default_params(flux_prec=1, **kw))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev())
    Fd = torch.zeros(npts, 5, dtype=torch.float64, device=dev())
    Ftd = torch.zeros_like(Fd)
    Sd = torch.zeros(npts, 4, 5, dtype=torch.float64, device=dev())
    K().cgks_flux(ctx, t(ql), t(gl), t(qr), t(gr), t(nrm), t(np.array([0.013])), Fd, Ftd, Sd)
    torch.cuda.synchronize()
    assert K().cgks_check(ctx) == (0, 0)
    for a, b in ((Fd, F), (Ftd, Ft), (Sd, S)):
        err = np.abs(a.cpu().numpy() - b).max() / np.abs(b).max()
        assert err <= 2e-5, err
    ctx.close()


# Unit roundoff of the split representation x = hi + lo: FP32 pairs carry 48 significand bits,
# but the operands start from FP64 values rounded once to FP32 and the products are summed in
# FP32, so FP32x3 is accurate to ~2^-24; a BF16 pair carries 16 bits (2^-17 after the dropped
# lo*lo term), FP32 accumulation below that.
U_SPLIT = {1: 2.0 ** -24, 2: 2.0 ** -17}


@pytest.mark.parametrize("recon_prec", [1, 2], ids=["fp32x3", "bf16x3"])
def test_split_reconstruction_accuracy(recon_prec):
    """Gauss-point values and gradients of the split-precision reconstruction against the FP64
    oracle.  The reconstruction is linear in the stencil data b (differences to the cell average
    and gradients) apart from the weights, so its error is bounded by ||E R||_inf * u * ||b||:
    measured relative to the size of the deviations from the cell average (values) and of the
    gradients, with ||E R||_inf <= 64 on the standard cell."""
    n = (17, 12, 10)
    nodes = W.perturbed_nodes(n, amp=0.05)
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.3), GAM)
    cells = np.arange(Q.shape[1])
    ref = O.recon(n, nodes.numpy(), O.params(), Q.numpy(), G.numpy(), L.numpy(), cells)
    ctx = K().Context([n], [nodes], K().default_params(recon_prec=recon_prec))
    gp = torch.zeros(Q.shape[1], 24, 5, 4, dtype=torch.float64, device=dev())
    K().cgks_recon(ctx, Q.to(dev()), G.to(dev()), L.to(dev()), gp)
    torch.cuda.synchronize()
    assert K().cgks_check(ctx) == (0, 0)
    out = gp.cpu().numpy()
    q0 = Q.numpy().T[:, None, :]
    tol = 64 * U_SPLIT[recon_prec]
    for v in range(5):
        dv = ref[:, :, v, 0] - q0[:, :, v]
        err = np.abs(out[:, :, v, 0] - ref[:, :, v, 0]).max() / max(np.abs(dv).max(), 1e-300)
        print("value", v, err)
        assert err <= tol, (v, err)
        for c in range(1, 4):
            err = np.abs(out[:, :, v, c] - ref[:, :, v, c]).max() / max(np.abs(ref[:, :, v, 1:]).max(), 1e-300)
            print("grad", v, c, err)
            assert err <= tol, (v, c, err)
    ctx.close()


@pytest.mark.parametrize("recon_prec,flux_prec", [(1, 0), (0, 1), (1, 1), (2, 0), (2, 1)])
def test_mixed_precision_tgv_error_vs_fp64(recon_prec, flux_prec):
    n = (20, 18, 16)
    nodes = W.perturbed_nodes(n, amp=0.05)
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.1), GAM)
    p0 = 1.0 / (GAM * 0.01)
    kw = dict(viscous=1, visc_law=1, mu0=1.0 / 1600, T_ref=p0, S_suth=p0 * 110.4 / 288.15, Pr=0.72, prandtl_fix=1)
    sto, Qo, Go, Lo, dto, _ = O.run(n, nodes.numpy(), O.params(**kw), Q.numpy(), G.numpy(), L.numpy(), 4)
    assert sto == 0
    ctx = K().Context([n], [nodes], K().default_params(recon_prec=recon_prec, flux_prec=flux_prec, **kw))
    Qd, Gd, Ld = Q.to(dev()), G.to(dev()), L.to(dev())
    dtd = torch.zeros(1, dtype=torch.float64, device=dev())
    for _ in range(4):
        K().cgks_step(ctx, Qd, Gd, Ld, dtd, use_cfl=True)
    torch.cuda.synchronize()
    assert K().cgks_check(ctx) == (0, 0)
    Qg = Qd.cpu().numpy()
    # relative L2 of density, velocity magnitude and total energy
    rho_e = np.linalg.norm(Qg[0] - Qo[0]) / np.linalg.norm(Qo[0])
    u = lambda q: np.sqrt(q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]
    u_e = np.linalg.norm(u(Qg) - u(Qo)) / np.linalg.norm(u(Qo))
    E_e = np.linalg.norm(Qg[4] - Qo[4]) / np.linalg.norm(Qo[4])
    assert max(rho_e, u_e, E_e) <= 1e-5, (rho_e, u_e, E_e)
    ctx.close()
