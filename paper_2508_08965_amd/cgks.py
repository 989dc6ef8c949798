"""Python binding of the CGKS-5 C ABI (include/cgks.h).

Argument marshalling only: every step of the path runs in the HIP library
``paper_2508_08965_amd/lib/libcgks.so``.  Device arrays are torch tensors (float64,
contiguous, on the context's device); streams are torch.cuda streams.  There is no CPU
fallback: if the library is missing or a call fails, a RuntimeError is raised.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libcgks.so")

OK, EINVAL, EHIP, ENOMEM, ENONPHYS, EUNSUPPORTED = 0, -1, -2, -3, -4, -5


class Params(C.Structure):
    """Mirror of cgks_params."""

    _fields_ = [
        ("gamma", C.c_double), ("cfl", C.c_double), ("tau_eps", C.c_double), ("tau_C", C.c_double),
        ("mu0", C.c_double), ("T_ref", C.c_double), ("S_suth", C.c_double), ("Pr", C.c_double),
        ("geno_C", C.c_double), ("geno_eps", C.c_double), ("geno_r", C.c_double),
        ("viscous", C.c_int), ("visc_law", C.c_int), ("tau_zero", C.c_int), ("linear", C.c_int),
        ("prandtl_fix", C.c_int), ("recon_prec", C.c_int), ("flux_prec", C.c_int), ("recon_impl", C.c_int),
        ("per_block", C.c_int), ("weights", C.c_int), ("jump_thresh", C.c_double), ("bc", C.c_int * 6),
        ("farfield", C.c_double * 5), ("positivity", C.c_int), ("pos_eps", C.c_double),
    ]


class Launch(C.Structure):
    """Mirror of cgks_launch."""

    _fields_ = [("tile_cells", C.c_int), ("ngroups", C.c_int), ("xcd", C.c_int), ("brick_y", C.c_int),
                ("brick_z", C.c_int), ("stage", C.c_int)]


_lib = None


def lib():
    """Load libcgks.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.cgks_default_params.argtypes = [C.POINTER(Params)]
        L.cgks_ctx_create.argtypes = [C.POINTER(vp), C.c_int, ip, C.POINTER(dp), C.POINTER(Params), vp]
        L.cgks_ctx_destroy.argtypes = [vp]
        L.cgks_num_cells.argtypes = [vp]
        L.cgks_num_cells.restype = C.c_long
        L.cgks_dt.argtypes = [vp, vp, vp, vp]
        L.cgks_dt_noalloc.argtypes = [vp, vp, vp, vp]
        L.cgks_diagnostics.argtypes = [vp, vp, vp, vp, vp]
        L.cgks_qcriterion.argtypes = [vp, vp, vp, vp, vp]
        L.cgks_diagnostics_hq.argtypes = [vp, vp, vp, vp, vp, vp]
        L.cgks_stage.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp]
        L.cgks_step.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp]
        L.cgks_check.argtypes = [vp, ip]
        L.cgks_recon.argtypes = [vp, vp, vp, vp, vp, vp]
        L.cgks_flux.argtypes = [vp, C.c_long, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.cgks_metrics.argtypes = [vp, vp, vp, vp, vp, vp]
        L.cgks_profile.argtypes = [vp, C.c_int]
        L.cgks_profile_read.argtypes = [vp, dp, C.POINTER(C.c_long)]
        L.cgks_get_launch.argtypes = [vp, C.c_int, C.POINTER(Launch)]
        L.cgks_set_launch.argtypes = [vp, C.c_int, C.POINTER(Launch)]
        L.cgks_autotune.argtypes = [vp, vp, vp, vp, vp, C.c_int, dp, C.c_int, vp]
        L.cgks_step_graph.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp]
        fp = C.POINTER(C.c_float)
        L.cgks_mlp_init.argtypes = [vp, C.c_ulonglong]
        L.cgks_mlp_set.argtypes = [vp, fp, C.c_int]
        L.cgks_mlp_get.argtypes = [vp, fp, C.c_int]
        L.cgks_mlp_grad.argtypes = [vp, vp, vp, C.c_long, vp, vp, vp]
        L.cgks_mlp_train.argtypes = [vp, vp, vp, C.c_long, C.c_int, C.c_int, C.c_float, fp, vp]
        L.cgks_mlp_infer.argtypes = [vp, vp, C.c_long, vp, vp]
        L.cgks_weights.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.cgks_mlp_fallback.argtypes = [vp, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]
        L.cgks_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def last_error() -> str:
    return lib().cgks_last_error().decode()


def _check(st, what):
    if st != OK:
        raise RuntimeError(f"{what} failed with status {st}: {last_error()}")


def default_params(**kw) -> Params:
    p = Params()
    lib().cgks_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        if k == "bc":
            v = (C.c_int * 6)(*v)
        elif k == "farfield":
            v = (C.c_double * 5)(*v)
        setattr(p, k, v)
    return p


def _ptr(t, numel=None, what="array"):
    """Device pointer of a contiguous float64 CUDA tensor; with numel, its size is checked on the
    host so that no kernel reads or writes past it."""
    if t is None:
        return None
    import torch
    if t.dtype != torch.float64 or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError("device arrays must be contiguous float64 CUDA tensors")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{what} has {t.numel()} elements, needs {numel}")
    return C.c_void_p(t.data_ptr())


def _state(ctx, Q, G, L, dt_dev=None):
    n = ctx.ncells
    return (_ptr(Q, 5 * n, "Q"), _ptr(G, 15 * n, "G"), _ptr(L, 60 * n, "L"),
            None if dt_dev is None else _ptr(dt_dev, 1, "dt"))


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Context:
    """A cgks_ctx: mesh, metrics, constant matrices and work buffers of one or more blocks."""

    def __init__(self, dims, nodes, params: Params, stream=None):
        import numpy as np
        dims = [tuple(int(x) for x in d) for d in dims]
        self._nodes = [np.ascontiguousarray(n.cpu().numpy() if hasattr(n, "cpu") else n, dtype=np.float64)
                       for n in nodes]
        flat = (C.c_int * (3 * len(dims)))(*[x for d in dims for x in d])
        ptrs = (C.POINTER(C.c_double) * len(dims))(*[a.ctypes.data_as(C.POINTER(C.c_double))
                                                     for a in self._nodes])
        h = C.c_void_p()
        _check(lib().cgks_ctx_create(C.byref(h), len(dims), flat, ptrs, C.byref(params), _stream(stream)),
               "cgks_ctx_create")
        self.h = h
        self.params = params
        self.dims = dims
        self.ncells = int(lib().cgks_num_cells(h))

    def close(self):
        if getattr(self, "h", None):
            lib().cgks_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cgks_dt(ctx: Context, Q, dt_dev, stream=None):
    _check(lib().cgks_dt(ctx.h, _ptr(Q, 5 * ctx.ncells, "Q"), _ptr(dt_dev, 1, "dt"), _stream(stream)), "cgks_dt")


def cgks_dt_noalloc(ctx: Context, Q, dt_dev, stream=None):
    """cgks_dt with its partial minima in the library's static device array (no allocation)."""
    _check(lib().cgks_dt_noalloc(ctx.h, _ptr(Q, 5 * ctx.ncells, "Q"), _ptr(dt_dev, 1, "dt"), _stream(stream)),
           "cgks_dt_noalloc")


def cgks_diagnostics(ctx: Context, Q, G, out, stream=None):
    """Flow diagnostics into the 6-element device tensor out: E_k, eps_S, mean rho, mean rho E,
    min rho, min p (asynchronous)."""
    n = ctx.ncells
    _check(lib().cgks_diagnostics(ctx.h, _ptr(Q, 5 * n, "Q"), _ptr(G, 15 * n, "G"), _ptr(out, 6, "out"),
                                  _stream(stream)), "cgks_diagnostics")


DIAG_NAMES = ("Ek", "epsS", "rho_mean", "rhoE_mean", "rho_min", "p_min")


def cgks_diagnostics_hq(ctx: Context, Q, G, L, out, stream=None):
    """E_k, eps_S, mean rho, mean rho E, min rho, min p (6 doubles into out) by 3^3 Gauss points
    per cell on the compact reconstruction."""
    q, g, l, _ = _state(ctx, Q, G, L)
    _check(lib().cgks_diagnostics_hq(ctx.h, q, g, l, _ptr(out, 6, "out"), _stream(stream)), "cgks_diagnostics_hq")


def cgks_qcriterion(ctx: Context, Q, G, out, stream=None):
    """Q-criterion of every cell into the device tensor out [N] (float64)."""
    _check(lib().cgks_qcriterion(ctx.h, _ptr(Q, 5 * ctx.ncells, "Q"), _ptr(G, 15 * ctx.ncells, "G"),
                                 _ptr(out, ctx.ncells, "out"), _stream(stream)), "cgks_qcriterion")


def cgks_stage(ctx: Context, stage: int, dt_dev, Q, G, L, stream=None):
    q, g, l, d = _state(ctx, Q, G, L, dt_dev)
    _check(lib().cgks_stage(ctx.h, int(stage), d, q, g, l, _stream(stream)), "cgks_stage")


def cgks_step(ctx: Context, Q, G, L, dt_dev, use_cfl=True, stream=None):
    q, g, l, d = _state(ctx, Q, G, L, dt_dev)
    _check(lib().cgks_step(ctx.h, q, g, l, d, int(bool(use_cfl)), _stream(stream)), "cgks_step")


def cgks_check(ctx: Context):
    """Returns (status, flags) without raising."""
    f = C.c_int(0)
    st = lib().cgks_check(ctx.h, C.byref(f))
    return st, f.value


def cgks_recon(ctx: Context, Q, G, L, gp, stream=None):
    q, g, l, _ = _state(ctx, Q, G, L)
    _check(lib().cgks_recon(ctx.h, q, g, l, _ptr(gp, 480 * ctx.ncells, "gp"), _stream(stream)), "cgks_recon")


def cgks_flux(ctx: Context, ql, gl, qr, gr, nrm, dt_dev, F, Ft, sides, stream=None):
    n = ql.shape[0]
    _check(lib().cgks_flux(ctx.h, n, _ptr(ql, 5 * n, "ql"), _ptr(gl, 15 * n, "gl"), _ptr(qr, 5 * n, "qr"),
                           _ptr(gr, 15 * n, "gr"), _ptr(nrm, 3 * n, "nrm"), _ptr(dt_dev, 1, "dt"),
                           _ptr(F, 5 * n, "F"), _ptr(Ft, 5 * n, "Ft"), _ptr(sides, 20 * n, "sides"),
                           _stream(stream)), "cgks_flux")


def cgks_metrics(ctx: Context, vol=None, J0=None, fn=None, fw=None, stream=None):
    n = ctx.ncells
    _check(lib().cgks_metrics(ctx.h, _ptr(vol, n, "vol"), _ptr(J0, 9 * n, "J0"), _ptr(fn, 36 * n, "fn"),
                              _ptr(fw, 12 * n, "fw"), _stream(stream)), "cgks_metrics")


KERNEL_KINDS = ("dt", "reconstruction", "flux_s1", "update_s1", "flux_s2", "update_s2")


def cgks_profile(ctx: Context, enable: bool):
    _check(lib().cgks_profile(ctx.h, int(bool(enable))), "cgks_profile")


def cgks_profile_read(ctx: Context):
    """{kind: (total ms, launches)} since the last read (synchronises)."""
    ms = (C.c_double * len(KERNEL_KINDS))()
    n = (C.c_long * len(KERNEL_KINDS))()
    _check(lib().cgks_profile_read(ctx.h, ms, n), "cgks_profile_read")
    return {k: (ms[i], n[i]) for i, k in enumerate(KERNEL_KINDS)}


KIND_NAMES = {1: "reconstruction", 2: "flux", 3: "update"}


def cgks_get_launch(ctx: Context, kind: int) -> dict:
    c = Launch()
    _check(lib().cgks_get_launch(ctx.h, kind, C.byref(c)), "cgks_get_launch")
    return {"tile_cells": c.tile_cells, "ngroups": c.ngroups, "xcd": c.xcd, "brick_y": c.brick_y,
            "brick_z": c.brick_z, "stage": c.stage}


def cgks_set_launch(ctx: Context, kind: int, tile_cells: int, ngroups: int, xcd: int, brick_y=0, brick_z=0,
                    stage=0):
    c = Launch(tile_cells, ngroups, xcd, brick_y, brick_z, stage)
    _check(lib().cgks_set_launch(ctx.h, kind, C.byref(c)), "cgks_set_launch")


def cgks_autotune(ctx: Context, Q, G, L, dt_dev, reps=3, stream=None):
    """Run the autotuner; returns the timed candidates as a list of dicts."""
    n = 1 + 7 * 128
    rep = (C.c_double * n)()
    q, g, l, d = _state(ctx, Q, G, L, dt_dev)
    _check(lib().cgks_autotune(ctx.h, q, g, l, d, reps, rep, n, _stream(stream)), "cgks_autotune")
    out = []
    for i in range(int(rep[0])):
        k, t, g, x, by, bz, ms = rep[1 + 7 * i: 8 + 7 * i]
        out.append({"kind": KIND_NAMES[int(k)], "tile_cells": int(t), "ngroups": int(g), "xcd": int(x),
                    "brick_y": int(by), "brick_z": int(bz), "ms": ms})
    return out


def cgks_step_graph(ctx: Context, Q, G, L, dt_dev, use_cfl=True, stream=None):
    q, g, l, d = _state(ctx, Q, G, L, dt_dev)
    _check(lib().cgks_step_graph(ctx.h, q, g, l, d, 1 if use_cfl else 0, _stream(stream)), "cgks_step_graph")


# ---- learned blend weights -------------------------------------------------------------------
MLP_PARAMS = 839


def _fptr(t):
    import torch
    if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError("feature/target arrays must be contiguous float32 CUDA tensors")
    return C.c_void_p(t.data_ptr())


def cgks_mlp_init(ctx: Context, seed: int):
    _check(lib().cgks_mlp_init(ctx.h, seed), "cgks_mlp_init")


def cgks_mlp_set(ctx: Context, w):
    import numpy as np
    a = np.ascontiguousarray(w, dtype=np.float32)
    _check(lib().cgks_mlp_set(ctx.h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size), "cgks_mlp_set")


def cgks_mlp_get(ctx: Context):
    import numpy as np
    a = np.zeros(MLP_PARAMS, dtype=np.float32)
    _check(lib().cgks_mlp_get(ctx.h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size), "cgks_mlp_get")
    return a


def _pairs(X, T):
    if X.dim() != 2 or X.shape[1] != 18 or T.dim() != 2 or T.shape[1] != 7 or T.shape[0] != X.shape[0]:
        raise ValueError("X must be [n, 18] and T [n, 7]")


def cgks_mlp_grad(ctx: Context, X, T, grad, loss, stream=None):
    _pairs(X, T)
    if grad.numel() < MLP_PARAMS or loss.numel() < 1:
        raise ValueError("grad needs 839 floats and loss 1")
    _check(lib().cgks_mlp_grad(ctx.h, _fptr(X), _fptr(T), X.shape[0], _fptr(grad), _fptr(loss), _stream(stream)),
           "cgks_mlp_grad")


def cgks_mlp_train(ctx: Context, X, T, steps, batch, lr, history=True, stream=None):
    import numpy as np
    _pairs(X, T)
    hist = np.zeros(max(steps, 1), dtype=np.float32) if history else None
    hp = hist.ctypes.data_as(C.POINTER(C.c_float)) if history else None
    _check(lib().cgks_mlp_train(ctx.h, _fptr(X), _fptr(T), X.shape[0], steps, batch, lr, hp, _stream(stream)),
           "cgks_mlp_train")
    return hist[:steps] if history else None


def cgks_mlp_infer(ctx: Context, X, Y, stream=None):
    if X.dim() != 2 or X.shape[1] != 18:
        raise ValueError("X must be [n, 18]")
    _check(lib().cgks_mlp_infer(ctx.h, _fptr(X), X.shape[0], _ptr(Y, 7 * X.shape[0], "Y"), _stream(stream)),
           "cgks_mlp_infer")


def cgks_weights(ctx: Context, Q, G, L, X, Wt, jump=None, stream=None):
    """Features X [5N, 18] (float32), weights used Wt [5N, 7] (float64) and jump flags [N] (uint8)."""
    import torch
    n = ctx.ncells
    if tuple(X.shape) != (5 * n, 18) or tuple(Wt.shape) != (5 * n, 7):
        raise ValueError("X must be [5N, 18] and Wt [5N, 7]")
    if jump is not None and (jump.dtype != torch.uint8 or jump.numel() != n or not jump.is_contiguous()
                             or jump.device.type != "cuda"):
        raise ValueError("jump must be a contiguous uint8 CUDA tensor of N elements")
    jp = None if jump is None else C.c_void_p(jump.data_ptr())
    q, g, l, _ = _state(ctx, Q, G, L)
    _check(lib().cgks_weights(ctx.h, q, g, l, _fptr(X), _ptr(Wt), jp, _stream(stream)), "cgks_weights")


def cgks_mlp_fallback(ctx: Context):
    f, e = C.c_longlong(), C.c_longlong()
    _check(lib().cgks_mlp_fallback(ctx.h, C.byref(f), C.byref(e)), "cgks_mlp_fallback")
    return f.value, e.value
