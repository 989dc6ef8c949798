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
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GAM = 1.4
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}  # TFLOP/s, MI355X dense (FP64 vector and matrix: 78.6)

# Algorithmic work per unit:
#   flux: source-level operation count of the gas-kinetic flux per Gauss point (flux_opcount.cpp),
#         the method's work counted once per Gauss point: each side's own moments and slopes
#         twice (left and right), the work both lanes of a pair repeat (frame, pair sums,
#         equilibrium state and slopes, collision time, time integrals) once; one stage
#         evaluates 12 Gauss points per cell (3 owned faces x 4 points)
#   reconstruction: the products as the method writes them, per cell and stage, 5 variables x
#         2 flops x (34 x 72 for a = R b, 96 x 34 for the Gauss-point values and gradients E a,
#         and the two smoothness forms through their triangular factors, 34 x 35 / 2 +
#         31 x 32 / 2); also reported with the cell's reflection symmetry taken out (below)
FLUX_FLOP_PER_GP = 7733        # first stage: flux, its time derivative, one-sided values and rates
FLUX_FLOP_PER_GP_DERIV = 7498  # second stage: time derivatives only (the update reads nothing else)
# what the lane pairs issue (the shared work twice): the hardware's view, for context only
FLUX_ISSUED_PER_GP, FLUX_ISSUED_PER_GP_DERIV = 8240, 7950
RECON_FLOP_PER_CELL = 2 * 5 * (34 * 72 + 96 * 34 + 34 * 35 // 2 + 31 * 32 // 2)
# the same products with the reflection symmetry of the centred standard cell taken out (the
# FP64 kernel's formulation): each face pair's values and gradients from one even and one odd
# product (48 x 34 instead of 96 x 34, then 96 additions), smoothness forms block diagonal by
# parity class (106 + 94 instead of 595 + 496 terms)
RECON_FLOP_PER_CELL_SYMMETRIC = 2 * 5 * (34 * 72 + 48 * 34 + 106 + 94) + 5 * 96
# what the FP64 kernel issues per cell: 86 matrix instructions (2048 flops) per 16 columns of
# (cell, variable), and coefficients 32-33 of a = R b on the vector ALU
RECON_MFMA_FLOP_PER_CELL = 5 * 86 * 2048 // 16 + 2 * 5 * 2 * 72
# algorithmic HBM bytes per cell of the update (state, stash, metrics, face records) and per
# Gauss point of the flux (344 in; 240 out in stage 1, 120 in stage 2)
UPDATE_BYTES = {1: 4592, 2: 3112}
FLUX_BYTES_PER_GP = {1: 584, 2: 464}
COUNTERS = os.path.join(ROOT, "profiles", "counters_tgv256_fp64.md")


def source_digest():
    """sha256 over the library sources (csrc/*.hip, *.h, *.cpp, sorted by name)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2508_08965_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed hardware-counter summary (FETCH_SIZE and
    WRITE_SIZE scaled by a copy kernel of known size), or None if the summary is missing, was taken
    on another workload, or the library sources changed since it was taken."""
    try:
        text = open(COUNTERS).read()
        blob = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(blob)
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256") != source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["read_bytes"] + k["write_bytes"]


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


def merged(prof):
    """Kernel kinds with both stages' flux (and update) launches taken together: total ms,
    launches, and the algorithmic work of all those launches."""
    out = {}
    for k, (ms, n) in prof.items():
        base = k.split("_s")[0]
        m, c = out.get(base, (0.0, 0))
        out[base] = (m + ms, c + n)
    return out


def flux_work(prof, N):
    """Method flops of every flux launch in prof (stage-1 and stage-2 counts differ)."""
    return 12 * N * (FLUX_FLOP_PER_GP * prof.get("flux_s1", (0, 0))[1]
                     + FLUX_FLOP_PER_GP_DERIV * prof.get("flux_s2", (0, 0))[1])


def roofline(prof, N, peak_key, counters=False):
    kinds = {k: v for k, v in merged(prof).items() if v[1] > 0}
    dom = max(kinds, key=lambda k: kinds[k][0])
    avg_ms = kinds[dom][0] / kinds[dom][1]
    if dom == "flux":
        # the work of an average flux launch (the stages alternate)
        work = flux_work(prof, N) / kinds[dom][1]
        roof = {"bound": "alu", "peak": PEAK[peak_key]}
    elif dom == "reconstruction":
        work = RECON_FLOP_PER_CELL * N
        roof = {"bound": "mfma", "peak": PEAK[peak_key]}
    else:
        return {"kernel": dom, "avg_ms": avg_ms, "bound": None, "achieved": None, "peak": None, "unit": None,
                "frac": None, "traffic": None}
    roof.update({"achieved": work / (avg_ms * 1e-3) / 1e12, "unit": "TFLOP/s",
                 "traffic": measured_traffic(dom) if counters else None})
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof.update({"kernel": dom, "avg_ms": avg_ms, "work_per_launch": work})
    return roof


def kernel_table(prof, N, ms_per_step=None):
    """Every kernel kind of an FP64 step against its own roof: average launch time (HIP events),
    the algorithmic work per launch and the achieved fraction (FP64 matrix / vector peaks and
    8 TB/s HBM), the flux and the update per stage; then the whole step: its algorithmic flops
    against the FP64 peak."""
    hbm = 8.0  # TB/s
    out = {}
    for k, (ms, n) in prof.items():
        if n == 0:
            continue
        avg = ms / n
        stage = 2 if k.endswith("_s2") else 1
        if k == "reconstruction":
            w = RECON_FLOP_PER_CELL * N
            ws = RECON_FLOP_PER_CELL_SYMMETRIC * N
            out[k] = {"avg_ms": avg, "bound": "mfma", "tflops": w / avg / 1e9, "frac": w / avg / 1e9 / PEAK["fp64"],
                      "tflops_symmetric": ws / avg / 1e9, "frac_symmetric": ws / avg / 1e9 / PEAK["fp64"],
                      "issued_frac": RECON_MFMA_FLOP_PER_CELL * N / avg / 1e9 / PEAK["fp64"],
                      "algorithmic_gbps": (98 + 480) * 8 * N / avg / 1e6}
        elif k.startswith("flux"):
            w = (FLUX_FLOP_PER_GP if stage == 1 else FLUX_FLOP_PER_GP_DERIV) * 12 * N
            wi = (FLUX_ISSUED_PER_GP if stage == 1 else FLUX_ISSUED_PER_GP_DERIV) * 12 * N
            out[k] = {"avg_ms": avg, "bound": "alu", "tflops": w / avg / 1e9, "frac": w / avg / 1e9 / PEAK["fp64"],
                      "issued_frac": wi / avg / 1e9 / PEAK["fp64"],
                      "algorithmic_gbps": FLUX_BYTES_PER_GP[stage] * 12 * N / avg / 1e6,
                      "hbm_frac": FLUX_BYTES_PER_GP[stage] * 12 * N / avg / 1e9 / hbm}
        elif k.startswith("update"):
            b = UPDATE_BYTES[stage] * N
            out[k] = {"avg_ms": avg, "bound": "hbm", "algorithmic_gbps": b / avg / 1e6, "frac": b / avg / 1e9 / hbm}
        elif k == "dt":
            b = 17 * 8 * N
            out[k] = {"avg_ms": avg, "bound": "hbm", "algorithmic_gbps": b / avg / 1e6, "frac": b / avg / 1e9 / hbm}
    if ms_per_step:
        steps = max(prof.get("flux_s2", (0, 0))[1], 1)
        w = (RECON_FLOP_PER_CELL * N * prof.get("reconstruction", (0, 0))[1] + flux_work(prof, N)) / steps
        out["step"] = {"ms": ms_per_step, "flops": w, "tflops": w / ms_per_step / 1e9,
                       "frac_fp64": w / ms_per_step / 1e9 / PEAK["fp64"],
                       "kernel_ms": sum(v[0] for v in prof.values()) / steps}
    return out


def oracle_rate(O, dims, nodes, prm, Q, G, L, steps, nthreads=0):
    """Cell-updates/s of the oracle over `steps` S2O4 steps with its set-up (metrics, work
    arrays) excluded: the time of a zero-step call on the same mesh is subtracted."""
    ncell = dims[0] * dims[1] * dims[2]
    t0 = time.perf_counter()
    O.run(dims, nodes, prm, Q, G, L, 0, nthreads=nthreads)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    st, *_ = O.run(dims, nodes, prm, Q, G, L, steps, nthreads=nthreads)
    t_run = time.perf_counter() - t0
    return {"value": steps * ncell / (t_run - t_setup), "seconds": t_run - t_setup, "setup_seconds": t_setup,
            "status": st}


def cpu_baseline(W, kw):
    """The oracle as it is (C, OpenMP), timed on this host: a bounded sample of the headline
    workload on every thread (one step on the 128^3 mesh of the 20-step parity configuration),
    the same workload on one thread, and the 2D density wave in full."""
    from oracle import oracle as O
    cores = O.num_threads()
    m, ksteps = 128, 1
    ns = (m, m, m)
    nd = W.perturbed_nodes(ns, amp=0.05)
    Qs, Gs, Ls = W.initial_state(nd, W.taylor_green(Ma=0.1), GAM)
    r = oracle_rate(O, ns, nd.numpy(), O.params(**kw), Qs.numpy(), Gs.numpy(), Ls.numpy(), ksteps, nthreads=cores)
    cpu = {"value": r["value"], "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
           "sample": f"{ksteps} S2O4 steps (CFL dt + 2 stages each) of the same TGV workload on a {m}^3 "
                     f"perturbed mesh, {r['seconds']:.1f} s (mesh set-up, {r['setup_seconds']:.1f} s, excluded)",
           "status": r["status"]}
    # the 2D density wave (40 x 40, tau = 0, 10 steps) in full
    n2 = (40, 40, 1)
    nd2 = W.cartesian_nodes(n2, (0, 0, 0), (2, 2, 2.0 / 40))
    q2, g2, l2 = W.initial_state(nd2, W.density_wave(dim=2), GAM)
    r2 = oracle_rate(O, n2, nd2.numpy(), O.params(tau_zero=1), q2.numpy(), g2.numpy(), l2.numpy(), 10,
                     nthreads=cores)
    cpu["density_wave_2d_40x40_10_steps"] = {"value": r2["value"], "seconds": r2["seconds"], "cores": cores}
    # one thread: the same TGV workload on a 48^3 mesh, one step
    m1 = 48
    n1 = (m1, m1, m1)
    nd1 = W.perturbed_nodes(n1, amp=0.05)
    q1, g1, l1 = W.initial_state(nd1, W.taylor_green(Ma=0.1), GAM)
    r1 = oracle_rate(O, n1, nd1.numpy(), O.params(**kw), q1.numpy(), g1.numpy(), l1.numpy(), 1, nthreads=1)
    O.run(n1, nd1.numpy(), O.params(**kw), q1.numpy(), g1.numpy(), l1.numpy(), 0, nthreads=cores)  # restore
    cpu["single_thread"] = {"value": r1["value"], "unit": "cell-updates/s", "cores": 1,
                            "sample": f"1 S2O4 step of the TGV workload on a {m1}^3 perturbed mesh, "
                                      f"{r1['seconds']:.1f} s (set-up excluded)"}
    return cpu


def hit_kw():
    # isotropic turbulence: rho 1, p 1/gamma (T = 1/gamma), Re_lambda 72 at u' = 0.2887, lambda 0.5
    T0 = 1.0 / GAM
    return dict(viscous=1, visc_law=1, mu0=2.0e-3, T_ref=T0, S_suth=T0 * 110.4 / 288.15, Pr=0.72, prandtl_fix=1)


def bench_batching(K, W, torch, steps, warmup):
    """Multi-block workload: 24 uneven periodic curvilinear blocks (seeded sizes) of decaying
    isotropic turbulence (Mt 0.5, k0 4), FP64.  Per-block launches against one launch per
    kernel over all blocks, with default and autotuned tiles, eager and graph-replayed."""
    dev = torch.device("cuda:0")
    dims = W.multiblock_dims()
    N = sum(a * b * c for a, b, c in dims)
    nodes_h, Qs, Gs, Ls = [], [], [], []
    for b, n in enumerate(dims):
        nd = W.perturbed_nodes(n, amp=0.05, device=dev)
        q, g, l = W.initial_state(nd, W.isotropic_turbulence(64, k0=4.0, Mt=0.5, seed=8965 + b), GAM)
        Qs.append(q)
        Gs.append(g)
        Ls.append(l)
        nodes_h.append(nd.cpu())
        del nd
    Q0 = torch.cat(Qs, dim=1).contiguous()
    G0 = torch.cat(Gs, dim=2).contiguous()
    L0 = torch.cat(Ls, dim=2).contiguous()
    del Qs, Gs, Ls
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    out = {"workload": f"{len(dims)} periodic perturbed curvilinear blocks, sizes from seed 8965 in "
                       "[32,160]x[32,96]x[32,64], decaying isotropic turbulence Mt 0.5 k0 4 Re_lambda 72, FP64",
           "cells": N, "blocks": len(dims), "variants": []}

    def run(ctx, label, graph=False):
        Q, G, L = Q0.clone(), G0.clone(), L0.clone()
        step = K.cgks_step_graph if graph else K.cgks_step
        for _ in range(warmup):
            step(ctx, Q, G, L, dt, use_cfl=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step(ctx, Q, G, L, dt, use_cfl=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = K.cgks_check(ctx)
        out["variants"].append({"variant": label, "value": N * steps / el, "unit": "cell-updates/s",
                                "ms_per_step": 1e3 * el / steps, "device_flags": st[1]})
        return Q

    ctx = K.Context(dims, nodes_h, K.default_params(per_block=1, **hit_kw()))
    Qa = run(ctx, "per-block launches (3 kernels x 24 blocks per stage)")
    ctx.close()
    torch.cuda.empty_cache()
    ctx = K.Context(dims, nodes_h, K.default_params(**hit_kw()))
    Qb = run(ctx, "one launch per kernel over all blocks, default tiles")
    out["bitwise_equal_to_per_block"] = bool(torch.equal(Qa, Qb))
    del Qa, Qb
    K.cgks_dt(ctx, Q0, dt)
    tune = K.cgks_autotune(ctx, Q0, G0, L0, dt, reps=2)
    out["autotune"] = {"candidates": tune, "picked": {K.KIND_NAMES[k]: K.cgks_get_launch(ctx, k) for k in (1, 2, 3)}}
    run(ctx, "one launch per kernel over all blocks, autotuned")
    run(ctx, "one launch per kernel over all blocks, autotuned, HIP graph of dt + 2 stages", graph=True)

    def kernel_ns_per_cell(c, Q, G, L, ncell):
        """Per kernel kind, average launch time per cell (HIP events), over `steps` steps."""
        _, prof = timed_steps(K, c, Q, G, L, dt, steps)
        return {k: 1e6 * ms / max(n, 1) / ncell for k, (ms, n) in prof.items() if n}

    Q, G, L = Q0.clone(), G0.clone(), L0.clone()
    out["kernel_ns_per_cell"] = {"batched_24_blocks": kernel_ns_per_cell(ctx, Q, G, L, N)}
    # time between kernels: the step's wall time less its kernels' HIP-event times (all that one
    # persistent launch per stage could remove besides the kernels' own tails)
    el, prof = timed_steps(K, ctx, Q, G, L, dt, steps)
    kms = sum(v[0] for v in prof.values()) / steps
    out["between_kernels_ms_per_step"] = {"step_ms": 1e3 * el / steps, "kernels_ms": kms,
                                          "gap_ms": 1e3 * el / steps - kms,
                                          "launches_per_step": sum(v[1] for v in prof.values()) / steps}
    ctx.close()
    del Q, G, L
    torch.cuda.empty_cache()
    # the same flow on one cubic block of about the same number of cells: separates what the
    # flow costs (more cells with an active nonlinear blend than in the Taylor-Green vortex at
    # Ma 0.1) from what the batching costs
    m = int(round(N ** (1.0 / 3.0)))
    n1 = (m, m, m)
    nd = W.perturbed_nodes(n1, amp=0.05, device=dev)
    Q, G, L = W.initial_state(nd, W.isotropic_turbulence(64, k0=4.0, Mt=0.5, seed=8965), GAM)
    nd_h = nd.cpu()
    ctx = K.Context([n1], [nd_h], K.default_params(**hit_kw()))
    del nd
    for _ in range(warmup):
        K.cgks_step(ctx, Q, G, L, dt, use_cfl=True)
    torch.cuda.synchronize()
    Q0s, G0s, L0s = Q.clone(), G.clone(), L.clone()
    el, _ = timed_steps(K, ctx, Q, G, L, dt, steps)
    out["single_block_same_flow"] = {"cells": m ** 3, "dims": list(n1), "value": m ** 3 * steps / el,
                                     "unit": "cell-updates/s", "ms_per_step": 1e3 * el / steps,
                                     "device_flags": K.cgks_check(ctx)[1]}
    out["kernel_ns_per_cell"]["single_block_same_flow"] = kernel_ns_per_cell(ctx, Q, G, L, m ** 3)
    ctx.close()
    # the linear scheme (chi = 1 everywhere: every wave of the reconstruction takes one path)
    # on both layouts: the per-cell cost of the batching and the block shapes alone, apart from
    # the flow's share of cells with an active nonlinear blend, which the coarser small blocks
    # raise
    lin = {}
    for label, dl, nl, (q0, g0, l0), nc in (("batched_24_blocks", dims, nodes_h, (Q0, G0, L0), N),
                                            ("single_block", [n1], [nd_h], (Q0s, G0s, L0s), m ** 3)):
        c = K.Context(dl, nl, K.default_params(linear=1, **hit_kw()))
        q, g, l = q0.clone(), g0.clone(), l0.clone()
        for _ in range(warmup):
            K.cgks_step(c, q, g, l, dt, use_cfl=True)
        lin[label] = kernel_ns_per_cell(c, q, g, l, nc)
        c.close()
        del q, g, l
    out["kernel_ns_per_cell_linear_scheme"] = lin
    del Q, G, L, Q0s, G0s, L0s
    torch.cuda.empty_cache()
    return out


def bench_learned(K, W, torch, n_eval=256, n_train=64, eval_t=0.2, train_steps=1500):
    """Learned blend weights on supersonic isotropic turbulence (Mt 1.0, k0 8, Re_lambda 100),
    with the interface-state limiter (positivity = 1: local Mach numbers reach ~2.8, and without
    it the scheme meets a non-physical state once shocklets form, t ~ 0.09 at 64^3): pairs
    (features, GENO weights) from the FP64 scheme at n_train^3 (seeds 8967-8970, run to
    t = lambda/u'), balanced between chi < 0.99 and chi ~ 1; FP32 Adam training on the GPU;
    then n_eval^3 (seed 8966) advanced past the formation of shocklets (to t >= eval_t) with
    learned and with GENO weights, the same number of steps each."""
    import numpy as np
    dev = torch.device("cuda:0")
    T0 = 1.0 / GAM
    kw = dict(viscous=1, visc_law=1, mu0=1.44e-3, T_ref=T0, S_suth=T0 * 110.4 / 288.15, Pr=0.72, prandtl_fix=1,
              positivity=1)
    two_pi = 2.0 * math.pi
    t_end = 0.25 / 0.5774
    # ---- training pairs -------------------------------------------------------------------------
    m = (n_train,) * 3
    nodes_m = W.cartesian_nodes(m, hi=(two_pi,) * 3)
    Xs, Ts = [], []
    gen = K.Context([m], [nodes_m], K.default_params(**kw))
    N = n_train ** 3
    X = torch.zeros(N * 5, 18, dtype=torch.float32, device=dev)
    Wt = torch.zeros(N * 5, 7, dtype=torch.float64, device=dev)
    rng = torch.Generator(device="cpu").manual_seed(8965)
    runs = []
    for seed in (8967, 8968, 8969, 8970):
        Q, G, L = W.initial_state(nodes_m.to(dev), W.isotropic_turbulence(64, k0=8.0, Mt=1.0, seed=seed), GAM)
        dt = torch.zeros(1, dtype=torch.float64, device=dev)
        t, k, flags = 0.0, 0, 0
        while t < t_end and k < 400:
            K.cgks_step(gen, Q, G, L, dt, use_cfl=True)
            flags = K.cgks_check(gen)[1]
            if flags:
                break
            t += dt.item()
            k += 1
            if k % 5 == 0 or t >= t_end:
                K.cgks_weights(gen, Q, G, L, X, Wt)
                ok = torch.isfinite(X).all(1) & torch.isfinite(Wt).all(1)
                low = (ok & (Wt[:, 0] < 0.99)).nonzero().squeeze(1)
                high = (ok & (Wt[:, 0] >= 0.99)).nonzero().squeeze(1)
                take = min(len(low), len(high), 20000)
                if take == 0:
                    continue
                pick_l = low[torch.randperm(len(low), generator=rng)[:take].to(dev)]
                pick_h = high[torch.randperm(len(high), generator=rng)[:take].to(dev)]
                idx = torch.cat([pick_l, pick_h])
                Xs.append(X[idx].clone())
                Ts.append(Wt[idx].float())
        runs.append({"seed": seed, "steps": k, "t": t, "stopped_by_flags": int(flags)})
    gen.close()
    Xtr = torch.cat(Xs)
    Ttr = torch.cat(Ts)
    perm = torch.randperm(Xtr.shape[0], generator=rng).to(dev)
    Xtr, Ttr = Xtr[perm].contiguous(), Ttr[perm].contiguous()
    frac_low = float((Ttr[:, 0] < 0.99).float().mean())
    del Xs, Ts, X, Wt
    # ---- evaluation mesh and training ---------------------------------------------------------
    e = (n_eval,) * 3
    nodes_e = W.cartesian_nodes(e, hi=(two_pi,) * 3)
    ctx = K.Context([e], [nodes_e], K.default_params(weights=1, **kw))
    K.cgks_mlp_init(ctx, 8965)
    torch.cuda.synchronize()
    tt = time.perf_counter()
    hist = K.cgks_mlp_train(ctx, Xtr, Ttr, steps=train_steps, batch=4096, lr=1e-3)
    t_train = time.perf_counter() - tt
    Q0, G0, L0 = W.initial_state(nodes_e.to(dev), W.isotropic_turbulence(128, k0=8.0, Mt=1.0, seed=8966), GAM)
    Ne = n_eval ** 3
    dt = torch.zeros(1, dtype=torch.float64, device=dev)

    def run(c, nsteps=None):
        """Steps to t >= eval_t (or nsteps steps); the time per step is taken over all of them
        (the device scalar dt is read back every 10 steps only)."""
        Q, G, L = Q0.clone(), G0.clone(), L0.clone()
        K.cgks_step(c, Q, G, L, dt, use_cfl=True)
        torch.cuda.synchronize()
        Q.copy_(Q0)
        G.copy_(G0)
        L.copy_(L0)
        tsum = torch.zeros(1, dtype=torch.float64, device=dev)
        k = 0
        t0 = time.perf_counter()
        while (nsteps is None and k < 1000) or (nsteps is not None and k < nsteps):
            K.cgks_step(c, Q, G, L, dt, use_cfl=True)
            tsum += dt
            k += 1
            if k % 10 == 0 and tsum.item() >= eval_t and nsteps is None:  # both runs sync alike
                break
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return Q, el, K.cgks_check(c), k, tsum.item()

    K.cgks_mlp_fallback(ctx)
    Qm, el_m, st_m, eval_steps, t_m = run(ctx)
    flagged, examined = K.cgks_mlp_fallback(ctx)
    ctx.close()
    torch.cuda.empty_cache()
    plain = K.Context([e], [nodes_e], K.default_params(**kw))
    Qp, el_p, st_p, _, t_p = run(plain, eval_steps)
    plain.close()

    def errs(a, b):
        d = a - b
        return {"rel_l2": float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(b)),
                "rel_linf": float(d.abs().max() / b.abs().max())}

    speed = lambda q: torch.sqrt(q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]
    return {
        "workload": f"isotropic turbulence Mt 1.0 k0 8 Re_lambda 100, {n_eval}^3 periodic Cartesian, FP64, "
                    f"interface-state limiter on; MLP 18-32-7 trained on {Xtr.shape[0]} balanced pairs from "
                    f"{n_train}^3 runs (4 seeds, t <= {max(r['t'] for r in runs):.3f})",
        "train": {"steps": train_steps, "batch": 4096, "lr": 1e-3, "seconds": t_train,
                  "loss_first10": float(np.mean(hist[:10])), "loss_last100": float(np.mean(hist[-100:])),
                  "pairs": int(Xtr.shape[0]), "fraction_chi_below_0.99": frac_low, "generator_runs": runs},
        "learned": {"value": Ne * eval_steps / el_m, "unit": "cell-updates/s", "ms_per_step": 1e3 * el_m / eval_steps,
                    "fallback_fraction": flagged / max(examined, 1), "device_flags": st_m[1]},
        "geno": {"value": Ne * eval_steps / el_p, "unit": "cell-updates/s", "ms_per_step": 1e3 * el_p / eval_steps,
                 "device_flags": st_p[1]},
        "learned_vs_geno_after_steps": {"steps": eval_steps, "t_learned": t_m, "t_geno": t_p,
                                        "rho": errs(Qm[0], Qp[0]),
                                        "speed": errs(speed(Qm), speed(Qp)), "rhoE": errs(Qm[4], Qp[4])},
    }


def bench_percell(K, W, torch, kw, n=128, steps=3):
    """The paper's storage argument (Sec. 4) measured: the same TGV step with the shared
    standard-cell matrix (matrix cores) and with per-cell stored matrices (recon_impl 2: each
    cell's coefficient map and Gauss-point evaluation, 48,960 bytes per cell, read every
    stage).  n^3 is chosen so that the per-cell matrices fit in HBM (256^3 would need 821 GB)."""
    dev = torch.device("cuda:0")
    m = (n,) * 3
    N = n ** 3
    nodes = W.perturbed_nodes(m, amp=0.05, device=dev)
    Q0, G0, L0 = W.initial_state(nodes, W.taylor_green(Ma=0.1), GAM)
    nodes = nodes.cpu()
    res, finals = {}, {}
    for name, impl in (("shared", 0), ("per_cell", 2)):
        try:
            ctx = K.Context([m], [nodes], K.default_params(recon_impl=impl, **kw))
        except RuntimeError as e:
            res[name] = {"error": str(e)}
            continue
        Q, G, L = Q0.clone(), G0.clone(), L0.clone()
        dt = torch.zeros(1, dtype=torch.float64, device=dev)
        K.cgks_step(ctx, Q, G, L, dt, use_cfl=True)
        Q.copy_(Q0)
        G.copy_(G0)
        L.copy_(L0)
        torch.cuda.synchronize()
        K.cgks_profile_read(ctx)
        K.cgks_profile(ctx, True)
        t0 = time.perf_counter()
        for _ in range(steps):
            K.cgks_step(ctx, Q, G, L, dt, use_cfl=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = K.cgks_profile_read(ctx)
        K.cgks_profile(ctx, False)
        rms, rn = prof["reconstruction"]
        r_ms = rms / max(rn, 1)
        matrix_bytes = 48960 * N if impl == 2 else 0
        # algorithmic bytes of one reconstruction launch: the per-cell matrices (shared: the
        # 84 KB constant block, negligible), Q G L J0 J0^-T in, 480 Gauss-point values out
        alg = matrix_bytes + (98 + 480) * 8 * N
        res[name] = {"value": N * steps / el, "unit": "cell-updates/s", "ms_per_step": 1e3 * el / steps,
                     "reconstruction_ms": r_ms, "matrix_storage_bytes": matrix_bytes if impl == 2 else 83968,
                     "reconstruction_algorithmic_GBps": alg / (r_ms * 1e-3) / 1e9,
                     # time the algorithmic bytes alone take at the 8 TB/s HBM peak: a floor for
                     # any implementation of this storage scheme
                     "reconstruction_hbm_floor_ms": alg / 8e12 * 1e3,
                     "device_flags": K.cgks_check(ctx)[1]}
        finals[name] = Q.cpu()
        ctx.close()
        del Q, G, L
        torch.cuda.empty_cache()
    out = {"workload": f"taylor-green vortex Re1600 Ma0.1, {n}^3 periodic perturbed curvilinear mesh, FP64, "
                       f"{steps} steps", "cells": N, "variants": res}
    if len(finals) == 2:
        a, b = finals["per_cell"], finals["shared"]
        out["rel_l2_Q_per_cell_vs_shared"] = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        if "reconstruction_ms" in res.get("per_cell", {}):
            out["reconstruction_time_ratio"] = res["per_cell"]["reconstruction_ms"] / res["shared"]["reconstruction_ms"]
    return out


def bench_walls(K, W, torch, kw, n=256, steps=5, warmup=2, check_oracle=True):
    """Wall sides at the headline size: the Taylor-Green vortex in the box [0, pi]^3 (bounded by
    its own symmetry planes: the octant of the periodic vortex on [0, 2 pi]^3 at twice the
    resolution) on a curvilinear mesh whose sides stay planar, once with symmetry planes and
    once with no-slip adiabatic walls on every side.  The headline line is the same step on a
    periodic mesh of the same size."""
    import numpy as np
    dev = torch.device("cuda:0")
    m = (n,) * 3
    N = n ** 3
    nodes = W.wall_perturbed_nodes(m, device=dev)
    Q0, G0, L0 = W.initial_state(nodes, W.taylor_green(Ma=0.1), GAM)
    nodes = nodes.cpu()
    res = {}
    for name, bc in (("symmetry_planes", 1), ("noslip_walls", 2)):
        ctx = K.Context([m], [nodes], K.default_params(bc=(bc,) * 6, **kw))
        vol = torch.zeros(N, dtype=torch.float64, device=dev)
        K.cgks_metrics(ctx, vol=vol)
        Q, G, L = Q0.clone(), G0.clone(), L0.clone()
        dt = torch.zeros(1, dtype=torch.float64, device=dev)
        mass0, energy0 = float((vol * Q[0]).sum()), float((vol * Q[4]).sum())
        for _ in range(warmup):
            K.cgks_step(ctx, Q, G, L, dt, use_cfl=True)
        torch.cuda.synchronize()
        K.cgks_profile_read(ctx)
        elapsed, prof = timed_steps(K, ctx, Q, G, L, dt, steps)
        res[name] = {"value": N * steps / elapsed, "unit": "cell-updates/s", "ms_per_step": 1e3 * elapsed / steps,
                     "kernel_ms": {k: {"total_ms": v[0], "launches": v[1]} for k, v in prof.items()},
                     "mass_rel_drift": abs(float((vol * Q[0]).sum()) - mass0) / mass0,
                     "energy_rel_drift": abs(float((vol * Q[4]).sum()) - energy0) / energy0,
                     "device_flags": K.cgks_check(ctx)[1]}
        if check_oracle:
            # untimed: stage 1 from the initial state on corner and side cells against the oracle
            from oracle import oracle as O
            rng = np.random.default_rng(8965 + bc)
            sides = rng.integers(0, n, size=(24, 3))
            sides[np.arange(24), rng.integers(0, 3, size=24)] = rng.choice([0, n - 1], size=24)
            cells = np.unique(np.concatenate([sides[:, 0] + n * (sides[:, 1] + n * sides[:, 2]),
                                              [0, n - 1, N - n, N - 1]])).astype(np.int64)
            dt_fix = 3.5e-4 * 256 / n
            Qh, Gh, Lh = Q0.cpu().numpy(), G0.cpu().numpy(), L0.cpu().numpy()
            st, oq, og, ol = O.stage1_cells(m, nodes.numpy(), O.params(bc=(bc,) * 6, **kw), dt_fix, Qh, Gh, Lh,
                                            cells)
            del Qh, Gh, Lh
            Q.copy_(Q0)
            G.copy_(G0)
            L.copy_(L0)
            dt.fill_(dt_fix)
            K.cgks_stage(ctx, 1, dt, Q, G, L)
            torch.cuda.synchronize()
            ci = torch.from_numpy(cells).to(dev)
            rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
            res[name]["parity_vs_oracle"] = {
                "stage": 1, "cells": int(len(cells)), "oracle_status": int(st),
                "rel_l2_Q": rel(Q[:, ci].T.cpu().numpy(), oq),
                "rel_l2_G": rel(G[:, :, ci].permute(2, 0, 1).cpu().numpy(), og),
                "rel_l2_L": rel(L[:, :, ci].permute(2, 0, 1).cpu().numpy(), ol)}
        ctx.close()
        del Q, G, L, vol
        torch.cuda.empty_cache()
    return {"workload": f"taylor-green vortex Re1600 Ma0.1 in [0, pi]^3, {n}^3 curvilinear mesh with planar sides, "
                        f"FP64, {steps} steps after {warmup}", "cells": N, "variants": res}


def bench_supersonic_tgv(K, W, torch, n=128, t_end=10.0, Ma=1.25):
    """Robustness run of Sec. 5: the supersonic Taylor-Green vortex (Ma 1.25, Re 1600, Pr 0.7,
    Sutherland) with the nonlinear scheme on the paper's uniform n^3 mesh, to t_end, with the
    kinetic energy and enstrophy history from the library's diagnostics: cell-centre midpoint
    sums, and 3^3 Gauss points per cell on the compact reconstruction."""
    dev = torch.device("cuda:0")
    m = (n,) * 3
    nodes = W.cartesian_nodes(m, hi=(2.0 * math.pi,) * 3)
    Q, G, L = W.initial_state(nodes.to(dev), W.taylor_green(Ma=Ma), GAM)
    p0 = 1.0 / (GAM * Ma * Ma)
    kw = dict(viscous=1, visc_law=1, mu0=1.0 / 1600, T_ref=p0, S_suth=p0 * 110.4 / 288.15, Pr=0.7, prandtl_fix=1)
    ctx = K.Context([m], [nodes], K.default_params(**kw))
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    d = torch.zeros(6, dtype=torch.float64, device=dev)

    def diag():
        K.cgks_diagnostics(ctx, Q, G, d)
        return d.tolist()

    def diag_hq():
        K.cgks_diagnostics_hq(ctx, Q, G, L, d)
        return d.tolist()

    d0 = diag()
    hist = [[0.0] + d0[:2] + diag_hq()[:2]]
    rho_min, p_min = d0[4], d0[5]
    t, k, flags = 0.0, 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while t < t_end and k < 20000:
        K.cgks_step(ctx, Q, G, L, dt, use_cfl=True)
        t += dt.item()
        k += 1
        if k % 50 == 0 or t >= t_end:
            x = diag()
            rho_min, p_min = min(rho_min, x[4]), min(p_min, x[5])
            if k % 100 == 0 or t >= t_end:
                hist.append([t] + x[:2] + diag_hq()[:2])
            flags = K.cgks_check(ctx)[1]
            if flags:
                break
        if k % 500 == 0:
            print(f"supersonic TGV {n}^3: step {k}, t = {t:.3f}", file=sys.stderr, flush=True)
    el = time.perf_counter() - t0
    d1 = diag()
    ctx.close()
    torch.cuda.empty_cache()
    return {"workload": f"supersonic taylor-green vortex Ma {Ma} Re 1600 Pr 0.7 Sutherland, {n}^3 uniform periodic "
                        f"mesh, nonlinear CGKS-5 FP64, to t = {t_end}",
            "steps": k, "t": t, "seconds": el, "cell_updates_per_s": n ** 3 * k / el, "device_flags": flags,
            "min_rho": rho_min, "min_p_over_p0": p_min / p0,
            "mass_rel_drift": (d1[2] - d0[2]) / d0[2], "energy_rel_drift": (d1[3] - d0[3]) / d0[3],
            "history_t_Ek_epsS_EkGauss_epsSGauss": hist}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="cells per axis")
    ap.add_argument("--no-oracle", action="store_true", help="skip the sampled parity check and the CPU baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip the reduced-precision variant")
    ap.add_argument("--error-steps", type=int, default=50, help="steps for the variant error against FP64")
    ap.add_argument("--no-batching", action="store_true", help="skip the multi-block batching measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-weight measurement")
    ap.add_argument("--no-percell", action="store_true", help="skip the per-cell matrix storage measurement")
    ap.add_argument("--no-supersonic", action="store_true", help="skip the supersonic Taylor-Green robustness run")
    ap.add_argument("--no-walls", action="store_true", help="skip the wall-side measurement")
    ap.add_argument("--only", choices=["batching"], default=None,
                    help="run one leg alone and print its record (for profiling that workload)")
    ap.add_argument("--supersonic-n", type=int, default=128, help="cells per axis of the supersonic TGV run")
    ap.add_argument("--supersonic-t", type=float, default=10.0, help="end time of the supersonic TGV run")
    ap.add_argument("--dump-state", default=None,
                    help="write the initial state and parameters of the FP64 workload for cgks_runner, then exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device (reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2508_08965_amd import cgks as K
    from paper_2508_08965_amd import workloads as W

    dev = torch.device("cuda:0")
    if args.only == "batching":
        print(json.dumps({"batching": bench_batching(K, W, torch, args.steps, args.warmup)}))
        return
    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    n = (args.n,) * 3
    N = n[0] * n[1] * n[2]
    nodes = W.perturbed_nodes(n, amp=0.05, device=dev)
    Q0, G0, L0 = W.initial_state(nodes, W.taylor_green(Ma=0.1), GAM)
    nodes_h = nodes.cpu()
    del nodes
    kw = tgv_kw()
    if args.dump_state:
        import ctypes
        prm = K.default_params(**kw)
        with open(args.dump_state, "wb") as f:
            f.write(b"CGKSST01")
            f.write(np.array([n[0], n[1], n[2], ctypes.sizeof(prm)], dtype=np.int32).tobytes())
            f.write(bytes(prm))
            nodes_h.numpy().astype(np.float64).tofile(f)
            for t in (Q0, G0, L0):
                t.cpu().numpy().tofile(f)
        print(json.dumps({"dumped": args.dump_state, "cells": N}))
        return
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
    roof = roofline(prof, N, "fp64", counters=(args.n == 256))
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
                "error_vs_fp64": {"steps": ne, "reference": "GPU FP64 path at this size; its whole-state parity "
                                  "with the FP64 oracle is a GPU test at 128^3 x 20 steps and 64^3 x 50 steps "
                                  "(tests/test_gpu_fullsize.py)",
                                  "rho": errs(Qv[0], Qr[0]), "speed": errs(speed(Qv), speed(Qr)),
                                  "rhoE": errs(Qv[4], Qr[4])},
                "device_flags": v_status[1],
            })
            vctx.close()
            del Qv, Gv, Lv
            torch.cuda.empty_cache()
    else:
        ctx.close()

    # ---- multi-block batching ------------------------------------------------------------------
    batching = None
    if not args.no_batching:
        batching = bench_batching(K, W, torch, args.steps, args.warmup)

    # ---- learned blend weights -----------------------------------------------------------------
    learned = None
    if not args.no_learned:
        learned = bench_learned(K, W, torch)

    # ---- per-cell stored matrices against the shared standard-cell matrix --------------------
    percell = None
    if not args.no_percell:
        percell = bench_percell(K, W, torch, kw)

    # ---- wall sides (symmetry planes, no-slip walls) at the headline size -------------------
    walls = None
    if not args.no_walls:
        walls = bench_walls(K, W, torch, kw, n=args.n, steps=args.steps, warmup=args.warmup,
                            check_oracle=not args.no_oracle)

    # ---- supersonic Taylor-Green vortex: robustness of the nonlinear scheme ------------------
    supersonic = None
    if not args.no_supersonic:
        supersonic = bench_supersonic_tgv(K, W, torch, n=args.supersonic_n, t_end=args.supersonic_t)

    # ---- CPU baseline: the oracle on a bounded sample of the same workload ------------------
    cpu = None
    if not args.no_oracle:
        cpu = cpu_baseline(W, kw)

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
        "kernels": kernel_table(prof, N, ms_per_step),
        "parity_vs_oracle": parity,
        "variants": variants,
        "batching": batching,
        "learned_weights": learned,
        "per_cell_storage": percell,
        "walls": walls,
        "supersonic_tgv": supersonic,
        "cpu_baseline": cpu,
        "device_flags": flags,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
