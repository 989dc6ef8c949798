"""Throughput of the CGKS-5 S2O4 step on one MI355X.

Workload: 3D Navier-Stokes Taylor-Green vortex (Re 1600, Ma 0.1, Pr 0.72, Sutherland), 256^3
cells on the periodic perturbed curvilinear mesh x = xi + 0.05 sin(xi) sin(eta) sin(zeta) per
axis, nonlinear CGKS-5.  A step is the CFL time step plus both S2O4 stages (reconstruction,
gas-kinetic flux, update) over every cell.  Inputs are synthetic and resident in HBM before
the timed region.  `value` is the FP64 path; the reduced-precision variants (FP32x3 or BF16x3
split-precision reconstruction on the FP32 or BF16 matrix cores + FP32 flux, FP64 metrics and
accumulation) are timed beside it with their L2/Linf error against FP64 after 50 steps.

Prints one JSON line.  --gpus N > 1 is not supported (single-GPU build).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GAM = 1.4
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}  # TFLOP/s, MI355X dense (FP64 vector and matrix: 78.6)

# Algorithmic work per unit (see the measurement section of the design notes):
#   flux: source-level operation count of the gas-kinetic flux per Gauss point (flux_opcount.cpp);
#         one stage evaluates 12 Gauss points per cell (3 owned faces x 4 points)
#   reconstruction: the formulated dense products per cell and stage, 5 variables x
#         2 (34x72 + 34x34 + 31x34 + 96x34)  (a = R b, Cholesky factors, Gauss-point values)
FLUX_FLOP_PER_GP = 8454
RECON_FLOP_PER_CELL = 2 * 5 * (34 * 72 + 34 * 34 + 31 * 34 + 96 * 34)


def tgv_kw():
    p0 = 1.0 / (GAM * 0.1 * 0.1)
    return dict(viscous=1, visc_law=1, mu0=1.0 / 1600.0, T_ref=p0, S_suth=p0 * 110.4 / 288.15, Pr=0.72,
                prandtl_fix=1)


def timed_steps(K, ctx, Q, G, L, dt, steps):
    import torch
    K.cgks_profile(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        K.cgks_step(ctx, Q, G, L, dt, use_cfl=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    K.cgks_profile(ctx, False)
    return t1 - t0, K.cgks_profile_read(ctx)


def roofline(prof, N, peak_key):
    kinds = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max(kinds, key=lambda k: kinds[k][0])
    avg_ms = kinds[dom][0] / kinds[dom][1]
    if dom == "flux":
        work = FLUX_FLOP_PER_GP * 12 * N
        roof = {"bound": "alu", "peak": PEAK[peak_key]}
    elif dom == "reconstruction":
        work = RECON_FLOP_PER_CELL * N
        roof = {"bound": "mfma", "peak": PEAK[peak_key]}
    else:
        return {"kernel": dom, "avg_ms": avg_ms, "bound": None, "achieved": None, "peak": None, "unit": None,
                "frac": None, "traffic": None}
    roof.update({"achieved": work / (avg_ms * 1e-3) / 1e12, "unit": "TFLOP/s", "traffic": None})
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof.update({"kernel": dom, "avg_ms": avg_ms, "work_per_launch": work})
    return roof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="cells per axis")
    ap.add_argument("--no-oracle", action="store_true", help="skip the sampled parity check and the CPU baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip the reduced-precision variant")
    ap.add_argument("--error-steps", type=int, default=50, help="steps for the variant error against FP64")
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
    Q0, G0, L0 = W.initial_state(nodes, W.taylor_green(Ma=0.1), GAM)
    nodes_h = nodes.cpu()
    del nodes
    kw = tgv_kw()
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx = K.Context([n], [nodes_h], K.default_params(**kw))

    # ---- sampled parity of stage 1 against the FP64 oracle (untimed) -------------------
    parity = None
    if not args.no_oracle:
        from oracle import oracle as O
        rng = np.random.default_rng(8965)
        cells = np.sort(rng.choice(N, size=48, replace=False))
        dt_fix = 3.5e-4 * 256 / args.n
        Qh, Gh, Lh = Q0.cpu().numpy(), G0.cpu().numpy(), L0.cpu().numpy()
        st, oq, og, ol = O.stage1_cells(n, nodes_h.numpy(), O.params(**kw), dt_fix, Qh, Gh, Lh, cells)
        del Qh, Gh, Lh
        Q1, G1, L1 = Q0.clone(), G0.clone(), L0.clone()
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

    # ---- FP64 path ------------------------------------------------------------------------
    Q, G, L = Q0.clone(), G0.clone(), L0.clone()
    for _ in range(args.warmup):
        K.cgks_step(ctx, Q, G, L, dt, use_cfl=True)
    torch.cuda.synchronize()
    K.cgks_profile_read(ctx)
    elapsed, prof = timed_steps(K, ctx, Q, G, L, dt, args.steps)
    status, flags = K.cgks_check(ctx)
    ms_per_step = 1e3 * elapsed / args.steps
    value = N * args.steps / elapsed
    roof = roofline(prof, N, "fp64")
    del Q, G, L

    # ---- reduced-precision variants, and their error against FP64 after error_steps --------
    variants = None
    if not args.no_variants:
        ne = args.error_steps
        Qr, Gr, Lr = Q0.clone(), G0.clone(), L0.clone()
        for _ in range(ne):
            K.cgks_step(ctx, Qr, Gr, Lr, dt, use_cfl=True)
        torch.cuda.synchronize()
        del Gr, Lr
        ctx.close()
        torch.cuda.empty_cache()

        def errs(a, b):
            d = a - b
            return {"rel_l2": float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(b)),
                    "rel_linf": float(d.abs().max() / b.abs().max())}

        speed = lambda q: torch.sqrt(q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]
        variants = []
        for name, rp in (("recon FP32x3 (FP32 matrix cores, split precision)", 1),
                         ("recon BF16x3 (BF16 matrix cores, split precision)", 2)):
            vctx = K.Context([n], [nodes_h], K.default_params(recon_prec=rp, flux_prec=1, **kw))
            Qv, Gv, Lv = Q0.clone(), G0.clone(), L0.clone()
            for _ in range(args.warmup):
                K.cgks_step(vctx, Qv, Gv, Lv, dt, use_cfl=True)
            torch.cuda.synchronize()
            K.cgks_profile_read(vctx)
            v_elapsed, v_prof = timed_steps(K, vctx, Qv, Gv, Lv, dt, args.steps)
            Qv.copy_(Q0)
            Gv.copy_(G0)
            Lv.copy_(L0)
            for _ in range(ne):
                K.cgks_step(vctx, Qv, Gv, Lv, dt, use_cfl=True)
            torch.cuda.synchronize()
            v_status = K.cgks_check(vctx)
            v_value = N * args.steps / v_elapsed
            variants.append({
                "variant": name + " + flux FP32; metrics, dt and S2O4 accumulation FP64",
                "value": v_value, "unit": "cell-updates/s",
                "ms_per_step": 1e3 * v_elapsed / args.steps,
                "speedup_vs_fp64": v_value / value,
                "kernel_ms": {k: {"total_ms": v[0], "launches": v[1]} for k, v in v_prof.items()},
                "roofline": roofline(v_prof, N, "bf16" if rp == 2 else "fp32"),
                "error_vs_fp64": {"steps": ne, "reference": "GPU FP64 path (matches the oracle, see parity)",
                                  "rho": errs(Qv[0], Qr[0]), "speed": errs(speed(Qv), speed(Qr)),
                                  "rhoE": errs(Qv[4], Qr[4])},
                "device_flags": v_status[1],
            })
            vctx.close()
            del Qv, Gv, Lv
            torch.cuda.empty_cache()
    else:
        ctx.close()

    # ---- CPU baseline: the oracle on a bounded sample of the same workload ------------------
    cpu = None
    if not args.no_oracle:
        from oracle import oracle as O
        m = 64
        ns = (m, m, m)
        nd = W.perturbed_nodes(ns, amp=0.05)
        Qs, Gs, Ls = W.initial_state(nd, W.taylor_green(Ma=0.1), GAM)
        tc = time.perf_counter()
        st, *_ = O.run(ns, nd.numpy(), O.params(**kw), Qs.numpy(), Gs.numpy(), Ls.numpy(), 2)
        tc = time.perf_counter() - tc
        cpu = {"value": 2 * m ** 3 / tc, "unit": "cell-updates/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"two S2O4 steps (CFL dt + 2 stages each) of the same TGV workload on a {m}^3 perturbed "
                         f"mesh, {tc:.1f} s", "status": st}

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
        "variants": variants,
        "cpu_baseline": cpu,
        "device_flags": flags,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
