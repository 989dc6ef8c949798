"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The GPU library never does.

The shared object is built from ``oracle/cgks_oracle.c`` with gcc and OpenMP,
in plain IEEE double precision (no fast-math, no FMA contraction).  A second build of the
same source, ``liboracle_fma.so``, lets the compiler fuse multiply-adds (``-mfma
-ffp-contract=fast``): an equally valid FP64 evaluation whose rounding differs.  The spread
between the two measures how far rounding alone moves a result, which sets the parity bar
of quantities formed by cancellation (the gradients and line derivatives).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cgks_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIBS = {"ieee": LIB, "fma": os.path.join(HERE, "liboracle_fma.so")}
_FLAGS = {"ieee": ["-ffp-contract=off"], "fma": ["-mfma", "-ffp-contract=fast"]}

OK, EINVAL, ENONPHYS = 0, -1, -4


class Params(C.Structure):
    """Mirror of ``or_params`` in cgks_oracle.c."""

    _fields_ = [
        ("gamma", C.c_double),
        ("cfl", C.c_double),
        ("tau_eps", C.c_double),
        ("tau_C", C.c_double),
        ("mu0", C.c_double),
        ("T_ref", C.c_double),
        ("S_suth", C.c_double),
        ("Pr", C.c_double),
        ("geno_C", C.c_double),
        ("geno_eps", C.c_double),
        ("geno_r", C.c_double),
        ("viscous", C.c_int),
        ("visc_law", C.c_int),
        ("tau_zero", C.c_int),
        ("linear", C.c_int),
        ("prandtl_fix", C.c_int),
        ("bc", C.c_int * 6),
        ("far", C.c_double * 5),
        ("positivity", C.c_int),
        ("pos_eps", C.c_double),
    ]


def params(**kw) -> Params:
    """Oracle parameters; defaults are the paper's constants (Sec. 3.3, Sec. 5)."""
    d = dict(gamma=1.4, cfl=0.5, tau_eps=0.05, tau_C=5.0, mu0=0.0, T_ref=1.0, S_suth=0.0,
             Pr=1.0, geno_C=150.0, geno_eps=1e-15, geno_r=2.0, viscous=0, visc_law=0,
             tau_zero=0, linear=0, prandtl_fix=0, bc=(0, 0, 0, 0, 0, 0), far=(1.0, 0.0, 0.0, 0.0, 2.5),
             positivity=0, pos_eps=1e-3)
    d.update(kw)
    d["bc"] = (C.c_int * 6)(*d["bc"])
    d["far"] = (C.c_double * 5)(*d["far"])
    return Params(**d)


def _stale(path):
    return not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC)


def build(force: bool = True) -> str:
    """Compile both oracle builds (gcc -O2 -fopenmp; IEEE double, and FMA-contracted)."""
    for variant, path in LIBS.items():
        if force or _stale(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp"] + _FLAGS[variant]
                                  + ["-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
            os.replace(tmp, path)
    return LIB


_libs = {}


def lib(variant: str = "ieee"):
    if variant not in _libs:
        path = LIBS[variant]
        if _stale(path):
            build(force=False)
        L = C.CDLL(path)
        dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_long)
        pp = C.POINTER(Params)
        L.oracle_constants.argtypes = [dp, dp, dp, dp, dp, dp, ip]
        L.oracle_metrics.argtypes = [ip, dp, dp, dp, dp, dp, dp]
        L.oracle_recon.argtypes = [ip, dp, pp, dp, dp, dp, lp, C.c_long, dp]
        L.oracle_flux.argtypes = [pp, C.c_long, dp, dp, dp, dp, dp, C.c_double, dp, dp, dp]
        L.oracle_positivity.argtypes = [pp, C.c_long, dp, dp, dp]
        L.oracle_nonreflecting_state.argtypes = [pp, dp, dp, dp]
        L.oracle_dt.argtypes = [ip, dp, pp, dp, dp]
        L.oracle_stage.argtypes = [ip, dp, pp, C.c_int, C.c_double, dp, dp, dp, dp, C.c_int]
        L.oracle_stage_weights.argtypes = [ip, dp, pp, C.c_int, C.c_double, dp, dp, dp, dp, dp]
        L.oracle_run.argtypes = [ip, dp, pp, dp, dp, dp, C.c_int, dp, dp, C.c_int]
        L.oracle_s2o4.argtypes = [C.c_long, C.c_double, dp, dp, dp, dp, dp, dp]
        L.oracle_stage1_cells.argtypes = [ip, dp, pp, C.c_double, dp, dp, dp, lp, C.c_long, dp, dp, dp]
        L.oracle_num_threads.restype = C.c_int
        L.oracle_mlp_forward.argtypes = [dp, C.c_long, dp, dp, dp]
        L.oracle_mlp_loss_grad.argtypes = [dp, C.c_long, dp, dp, dp, dp]
        L.oracle_adam.argtypes = [C.c_long, dp, dp, dp, dp, C.c_int, C.c_double, C.c_double, C.c_double,
                                  C.c_double]
        L.oracle_bf16.argtypes = [C.c_long, dp, dp]
        L.oracle_features.argtypes = [ip, dp, pp, dp, dp, lp, C.c_long, C.c_double, dp, ip]
        L.oracle_recon_weights.argtypes = [ip, dp, pp, dp, dp, dp, lp, C.c_long, dp, dp, dp]
        L.oracle_diagnostics.argtypes = [ip, dp, pp, dp, dp, dp]
        L.oracle_diagnostics_hq.argtypes = [ip, dp, pp, dp, dp, dp, dp]
        L.oracle_qcriterion.argtypes = [ip, dp, dp, dp]
        _libs[variant] = L
    return _libs[variant]


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _arr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _dims(dims):
    return (C.c_int * 3)(*[int(x) for x in dims])


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def constants():
    """R (34x72), EV (24x34), EG (24x3x34), GH, GL, GT (34x34), multi-indices (34x3)."""
    R = np.zeros((34, 72)); ev = np.zeros((24, 34)); eg = np.zeros((24, 3, 34))
    gh = np.zeros((34, 34)); gl = np.zeros((34, 34)); gt = np.zeros((34, 34))
    mi = np.zeros((34, 3), dtype=np.int32)
    lib().oracle_constants(_d(R), _d(ev), _d(eg), _d(gh), _d(gl), _d(gt),
                           mi.ctypes.data_as(C.POINTER(C.c_int)))
    return dict(R=R, EV=ev, EG=eg, GH=gh, GL=gl, GT=gt, MI=mi)


def metrics(dims, nodes):
    n = int(np.prod(dims))
    nodes = _arr(nodes)
    vol = np.zeros(n); J0 = np.zeros((n, 3, 3)); JiT = np.zeros((n, 3, 3))
    fn = np.zeros((n, 3, 4, 3)); fw = np.zeros((n, 3, 4))
    st = lib().oracle_metrics(_dims(dims), _d(nodes), _d(vol), _d(J0), _d(JiT), _d(fn), _d(fw))
    if st:
        raise ValueError(f"oracle_metrics status {st}")
    return dict(vol=vol, J0=J0, JinvT=JiT, fn=fn, fw=fw)


def recon(dims, nodes, prm, Q, G, L, cells, variant="ieee"):
    """Gauss-point values and physical gradients: [ncells, 24, 5, 4]."""
    nodes, Q, G, L = _arr(nodes), _arr(Q), _arr(G), _arr(L)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), 24, 5, 4))
    st = lib(variant).oracle_recon(_dims(dims), _d(nodes), C.byref(prm), _d(Q), _d(G), _d(L),
                            cells.ctypes.data_as(C.POINTER(C.c_long)), len(cells), _d(out))
    if st:
        raise ValueError(f"oracle_recon status {st}")
    return out


def flux(prm, ql, gl, qr, gr, nrm, dt):
    """GKS flux at independent points.  ql[n,5], gl[n,5,3], nrm[n,3] -> F, Ft [n,5], sides [n,4,5]."""
    ql, gl, qr, gr, nrm = map(_arr, (ql, gl, qr, gr, nrm))
    n = ql.shape[0]
    F = np.zeros((n, 5)); Ft = np.zeros((n, 5)); S = np.zeros((n, 4, 5))
    st = lib().oracle_flux(C.byref(prm), n, _d(ql), _d(gl), _d(qr), _d(gr), _d(nrm), float(dt),
                           _d(F), _d(Ft), _d(S))
    return st, F, Ft, S


def positivity(prm, qbar, q, g):
    """The interface-state limiter (reading D28) on independent states: qbar, q [n,5],
    g [n,5,3] -> limited (q, g) copies."""
    qbar = _arr(qbar)
    q, g = _arr(q).copy(), _arr(g).copy()
    st = lib().oracle_positivity(C.byref(prm), q.shape[0], _d(qbar), _d(q), _d(g))
    if st:
        raise ValueError(f"oracle_positivity status {st}")
    return q, g


def nonreflecting_state(prm, q, n):
    """Boundary state of a non-reflecting side (reading D29) for the interior state q [5] and
    the outward unit normal n [3]."""
    q, n = _arr(q), _arr(n)
    out = np.zeros(5)
    st = lib().oracle_nonreflecting_state(C.byref(prm), _d(q), _d(n), _d(out))
    if st:
        raise ValueError(f"oracle_nonreflecting_state status {st}")
    return out


def cfl_dt(dims, nodes, prm, Q):
    nodes, Q = _arr(nodes), _arr(Q)
    out = C.c_double(0)
    st = lib().oracle_dt(_dims(dims), _d(nodes), C.byref(prm), _d(Q), C.byref(out))
    if st:
        raise ValueError(f"oracle_dt status {st}")
    return out.value


def stage(dims, nodes, prm, s, dt, Q, G, L, stash, nthreads=0, variant="ieee"):
    """One stage in place on caller arrays (float64, C-contiguous)."""
    nodes = _arr(nodes)
    for a in (Q, G, L, stash):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    return lib(variant).oracle_stage(_dims(dims), _d(nodes), C.byref(prm), int(s), float(dt), _d(Q), _d(G),
                              _d(L), _d(stash), int(nthreads))


def stage_weights(dims, nodes, prm, s, dt, Q, G, L, stash, win, variant="ieee"):
    """One stage in place with given blend weights win [N, 5, 7] (chi, omega_1..6)."""
    nodes = _arr(nodes)
    win = _arr(win)
    for a in (Q, G, L, stash):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    assert win.size == 35 * Q.shape[1]
    return lib(variant).oracle_stage_weights(_dims(dims), _d(nodes), C.byref(prm), int(s), float(dt), _d(Q), _d(G),
                                             _d(L), _d(stash), _d(win))


def run(dims, nodes, prm, Q, G, L, nsteps, dt=0.0, nthreads=0, variant="ieee"):
    """nsteps S2O4 steps on copies; returns (status, Q, G, L, last dt, elapsed t)."""
    nodes = _arr(nodes)
    Q, G, L = _arr(Q).copy(), _arr(G).copy(), _arr(L).copy()
    d = C.c_double(float(dt))
    t = C.c_double(0)
    st = lib(variant).oracle_run(_dims(dims), _d(nodes), C.byref(prm), _d(Q), _d(G), _d(L), int(nsteps),
                          C.byref(d), C.byref(t), int(nthreads))
    return st, Q, G, L, d.value, t.value


def s2o4(dt, q, Ln, Ltn, Lts):
    q, Ln, Ltn, Lts = map(_arr, (q, Ln, Ltn, Lts))
    qs = np.zeros_like(q); qn = np.zeros_like(q)
    lib().oracle_s2o4(q.size, float(dt), _d(q), _d(Ln), _d(Ltn), _d(Lts), _d(qs), _d(qn))
    return qs, qn


def stage1_cells(dims, nodes, prm, dt, Q, G, L, cells, variant="ieee"):
    """Stage-1 outputs (Q*, G*, L*) of the listed cells only: [n,5], [n,5,3], [n,5,12]."""
    nodes, Q, G, L = _arr(nodes), _arr(Q), _arr(G), _arr(L)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    n = len(cells)
    oq = np.zeros((n, 5)); og = np.zeros((n, 5, 3)); ol = np.zeros((n, 5, 12))
    st = lib(variant).oracle_stage1_cells(_dims(dims), _d(nodes), C.byref(prm), float(dt), _d(Q), _d(G), _d(L),
                                   cells.ctypes.data_as(C.POINTER(C.c_long)), n, _d(oq), _d(og), _d(ol))
    return st, oq, og, ol


# ---- learned blend weights (MLP 18 -> 32 -> 7) --------------------------------------------
MLP_IN, MLP_H, MLP_OUT = 18, 32, 7
MLP_NPAR = MLP_H * MLP_IN + MLP_H + MLP_OUT * MLP_H + MLP_OUT


def mlp_forward(w, X):
    """Outputs [n, 7] (chi, omega_1..6) and hidden activations [n, 32] of the FP64 MLP."""
    w, X = _arr(w), _arr(X)
    n = X.shape[0]
    Y = np.zeros((n, MLP_OUT)); H = np.zeros((n, MLP_H))
    lib().oracle_mlp_forward(_d(w), n, _d(X), _d(Y), _d(H))
    return Y, H


def mlp_loss_grad(w, X, T):
    """Mean-square loss over the batch and its gradient [839]."""
    w, X, T = _arr(w), _arr(X), _arr(T)
    g = np.zeros(MLP_NPAR)
    loss = C.c_double(0)
    st = lib().oracle_mlp_loss_grad(_d(w), X.shape[0], _d(X), _d(T), C.byref(loss), _d(g))
    if st:
        raise ValueError(f"oracle_mlp_loss_grad status {st}")
    return loss.value, g


def adam(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on copies; returns (w, m, v)."""
    w, m, v, g = (_arr(a).copy() for a in (w, m, v, g))
    st = lib().oracle_adam(w.size, _d(w), _d(m), _d(v), _d(g), int(t), float(lr), float(b1), float(b2), float(eps))
    if st:
        raise ValueError(f"oracle_adam status {st}")
    return w, m, v


def bf16(x):
    """Round to BF16 (nearest, ties to even) through binary32."""
    x = _arr(x)
    out = np.zeros_like(x)
    lib().oracle_bf16(x.size, _d(x), _d(out))
    return out


def features(dims, nodes, prm, Q, L, cells, thresh=0.05):
    """MLP input features [ncells, 5, 18] and jump indicator [ncells] of the listed cells."""
    nodes, Q, L = _arr(nodes), _arr(Q), _arr(L)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    X = np.zeros((len(cells), 5, MLP_IN))
    jump = np.zeros(len(cells), dtype=np.int32)
    st = lib().oracle_features(_dims(dims), _d(nodes), C.byref(prm), _d(Q), _d(L),
                               cells.ctypes.data_as(C.POINTER(C.c_long)), len(cells), float(thresh), _d(X),
                               jump.ctypes.data_as(C.POINTER(C.c_int)))
    if st:
        raise ValueError(f"oracle_features status {st}")
    return X, jump.astype(bool)


def recon_weights(dims, nodes, prm, Q, G, L, cells, win=None):
    """Reconstruction of the listed cells with given blend weights win [ncells, 5, 7] (or GENO's
    if None); returns (gp [ncells, 24, 5, 4], weights used [ncells, 5, 7])."""
    nodes, Q, G, L = _arr(nodes), _arr(Q), _arr(G), _arr(L)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), 24, 5, 4))
    wout = np.zeros((len(cells), 5, 7))
    wp = None if win is None else _d(_arr(win))
    st = lib().oracle_recon_weights(_dims(dims), _d(nodes), C.byref(prm), _d(Q), _d(G), _d(L),
                                    cells.ctypes.data_as(C.POINTER(C.c_long)), len(cells), wp, _d(out), _d(wout))
    if st:
        raise ValueError(f"oracle_recon_weights status {st}")
    return out, wout


def diagnostics(dims, nodes, prm, Q, G):
    """Flow diagnostics of the Taylor-Green section (Sec. 5): midpoint-rule volume averages of
    the kinetic energy E_k and the enstrophy eps_S (normalised by the mean density and the
    domain volume), with the mean density and total energy and the minima of rho and p."""
    nodes, Q, G = _arr(nodes), _arr(Q), _arr(G)
    out = np.zeros(6)
    st = lib().oracle_diagnostics(_dims(dims), _d(nodes), C.byref(prm), _d(Q), _d(G), _d(out))
    if st:
        raise ValueError(f"oracle_diagnostics status {st}")
    return dict(Ek=out[0], epsS=out[1], rho_mean=out[2], rhoE_mean=out[3], rho_min=out[4], p_min=out[5])


def diagnostics_hq(dims, nodes, prm, Q, G, L):
    """The same diagnostics by 3^3-point Gauss quadrature of each cell, with the state and its
    velocity gradient from the cell's compact reconstruction (periodic blocks)."""
    nodes, Q, G, L = _arr(nodes), _arr(Q), _arr(G), _arr(L)
    out = np.zeros(6)
    st = lib().oracle_diagnostics_hq(_dims(dims), _d(nodes), C.byref(prm), _d(Q), _d(G), _d(L), _d(out))
    if st:
        raise ValueError(f"oracle_diagnostics_hq status {st}")
    return dict(Ek=out[0], epsS=out[1], rho_mean=out[2], rhoE_mean=out[3], rho_min=out[4], p_min=out[5])


def qcriterion(dims, Q, G):
    """Q-criterion of every cell, (|Omega|^2 - |S|^2) / 2 of the velocity gradient: [N]."""
    Q, G = _arr(Q), _arr(G)
    out = np.zeros(int(np.prod(dims)))
    st = lib().oracle_qcriterion(_dims(dims), _d(Q), _d(G), _d(out))
    if st:
        raise ValueError(f"oracle_qcriterion status {st}")
    return out
