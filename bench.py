"""Throughput of the CGKS-5 S2O4 step on one MI355X.

Workload: 3D Navier-Stokes Taylor-Green vortex (Re 1600, Ma 0.1, Pr 0.72, Sutherland), 256^3
cells on the periodic perturbed curvilinear mesh x = xi + 0.05 sin(xi) sin(eta) sin(zeta) per
axis, nonlinear CGKS-5, FP64.  A step is the CFL time step plus both S2O4 stages
(reconstruction, gas-kinetic flux, update) over every cell.  Inputs are synthetic and resident
in HBM before the timed region.

Prints one JSON line.  --gpus N > 1 is not supported (single-GPU build).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GAM = 1.4
PEAK_FP64_TFLOPS = 78.6  # MI355X vector / matrix FP64
PEAK_HBM_GBS = 8000.0

# Algorithmic work per unit, see the measurement section of the design notes.
FLUX_FLOP_PER_GP = None   # filled from the op count of the flux (per Gauss point)
RECON_FLOP_PER_CELL = 2 * 5 * (34 * 72 + 24 * 4 * 34 + 2 * 34 * 34)


def tgv_params(K, n_cells_axis):
    p0 = 1.0 / (GAM * 0.1 * 0.1)
    return K.default_params(viscous=1, visc_law=1, mu0=1.0 / 1600.0, T_ref=p0, S_suth=p0 * 110.4 / 288.15,
                            Pr=0.72, prandtl_fix=1)


def oracle_params(O):
    p0 = 1.0 / (GAM * 0.1 * 0.1)
    return O.params(viscous=1, visc_law=1, mu0=1.0 / 1600.0, T_ref=p0, S_suth=p0 * 110.4 / 288.15, Pr=0.72,
                    prandtl_fix=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="cells per axis")
    ap.add_argument("--no-oracle", action="store_true", help="skip the sampled parity check and the CPU baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2508_08965_amd import cgks as K
    from paper_2508_08965_amd import workloads as W

    dev = torch.device("cuda:0")
    n = (args.n,) * 3
    N = n[0] * n[1] * n[2]
    nodes = W.perturbed_nodes(n, amp=0.05, device=dev)
    Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.1), GAM)
    nodes_h = nodes.cpu()
    del nodes
    prm = tgv_params(K, args.n)
    ctx = K.Context([n], [nodes_h], prm)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)

    # ---- sampled parity of stage 1 against the FP64 oracle (untimed) -------------------
    parity = None
    if not args.no_oracle:
        from oracle import oracle as O
        rng = np.random.default_rng(8965)
        cells = np.sort(rng.choice(N, size=48, replace=False))
        dt_fix = 3.5e-4
        Qh, Gh, Lh = Q.cpu().numpy(), G.cpu().numpy(), L.cpu().numpy()
        st, oq, og, ol = O.stage1_cells(n, nodes_h.numpy(), oracle_params(O), dt_fix, Qh, Gh, Lh, cells)
        del Qh, Gh, Lh
        Q1, G1, L1 = Q.clone(), G.clone(), L.clone()
        dt.fill_(dt_fix)
        K.cgks_stage(ctx, 1, dt, Q1, G1, L1)
        torch.cuda.synchronize()
        ci = torch.from_numpy(cells).to(dev)
        gq = Q1[:, ci].T.cpu().numpy()
        gg = G1[:, :, ci].permute(2, 0, 1).cpu().numpy()
        gl = L1[:, :, ci].permute(2, 0, 1).cpu().numpy()
        del Q1, G1, L1
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        parity = {"stage": 1, "cells": int(len(cells)), "oracle_status": int(st),
                  "rel_l2_Q": rel(gq, oq), "rel_l2_G": rel(gg, og), "rel_l2_L": rel(gl, ol)}
        torch.cuda.empty_cache()

    # ---- warmup ---------------------------------------------------------------------------
    for _ in range(args.warmup):
        K.cgks_step(ctx, Q, G, L, dt, use_cfl=True)
    torch.cuda.synchronize()
    K.cgks_profile_read(ctx)

    # ---- timed region -----------------------------------------------------------------------
    K.cgks_profile(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        K.cgks_step(ctx, Q, G, L, dt, use_cfl=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    K.cgks_profile(ctx, False)
    prof = K.cgks_profile_read(ctx)
    status, flags = K.cgks_check(ctx)
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = N * args.steps / elapsed

    # dominant kernel and its roofline
    kinds = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max(kinds, key=lambda k: kinds[k][0])
    avg_ms = kinds[dom][0] / kinds[dom][1]
    if dom == "flux" and FLUX_FLOP_PER_GP:
        work = FLUX_FLOP_PER_GP * 12 * N
        roof = {"bound": "alu", "achieved": work / (avg_ms * 1e-3) / 1e12, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "traffic": None}
    elif dom == "reconstruction":
        work = RECON_FLOP_PER_CELL * N
        roof = {"bound": "alu", "achieved": work / (avg_ms * 1e-3) / 1e12, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "traffic": None}
    else:
        roof = {"bound": None, "achieved": None, "peak": None, "unit": None, "traffic": None}
    if roof.get("achieved"):
        roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = dom
    roof["avg_ms"] = avg_ms

    # ---- CPU baseline: the oracle on a bounded sample of the same workload ------------------
    cpu = None
    if not args.no_oracle:
        from oracle import oracle as O
        m = 64
        ns = (m, m, m)
        nd = W.perturbed_nodes(ns, amp=0.05)
        Qs, Gs, Ls = W.initial_state(nd, W.taylor_green(Ma=0.1), GAM)
        tc = time.perf_counter()
        st, *_ = O.run(ns, nd.numpy(), oracle_params(O), Qs.numpy(), Gs.numpy(), Ls.numpy(), 2)
        tc = time.perf_counter() - tc
        cpu = {"value": 2 * m ** 3 / tc, "unit": "cell-updates/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"two S2O4 steps (CFL dt + 2 stages each) of the same TGV workload on a {m}^3 perturbed mesh, "
                         f"{tc:.1f} s", "status": st}

    out = {
        "metric": "cell-updates/sec per S2O4 step at 256^3 TGV + L2 error vs FP64 oracle",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"taylor-green vortex Re1600 Ma0.1 Pr0.72, {n[0]}^3 periodic perturbed curvilinear "
                               "mesh (amp 0.05), nonlinear CGKS-5, FP64", "cells": N, "variant": "fp64"},
        "kernel_ms": {k: {"total_ms": v[0], "launches": v[1]} for k, v in prof.items()},
        "roofline": roof,
        "parity_vs_oracle": parity,
        "cpu_baseline": cpu,
        "device_flags": flags,
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
