"""Parity bars of the GPU path against the FP64 oracle (test helpers, no tests here).

Cell averages Q are held to the 1e-12 relative L2 bar.  Gradients G and line derivatives L
are differences of interface values (eqs. derivative and derivative-l): an interface value of
size |Q| is rounded at about 2^-53 |Q| by any FP64 evaluation, and G and L are small
differences of such values, so the agreement two correct FP64 evaluations can reach is set
by rounding, not by 1e-12 of the (small) result.  That floor is measured, not assumed: the
oracle is evaluated a second time, built with fused multiply-adds (an equally valid FP64
evaluation whose rounding differs) and fed inputs that differ from the given ones by at most
one unit in the last place each (``jitter``).  Per variable group (density, the momentum
vector, energy: the face-frame rotations mix the momentum components) the GPU must agree
with the oracle within

    max(1e-12 * rms(oracle), 2 * rms(second evaluation - oracle)).
"""
import numpy as np
import torch

from oracle import oracle as O

TOL = 1e-12
FACTOR = 2.0
GROUPS = {"rho": [0], "momentum": [1, 2, 3], "energy": [4]}


def as_np(a):
    return a.detach().cpu().numpy() if torch.is_tensor(a) else np.asarray(a)


def jitter(a, seed):
    """Each value moved to its next representable neighbour up or down, or kept (1/3 each).
    Row by row along the first axes, so that full-size states need little extra memory."""
    a = np.array(as_np(a), dtype=np.float64, order="C")
    rng = np.random.default_rng(seed)
    rows = a.reshape(-1, a.shape[-1])
    for row in rows:
        r = rng.integers(-1, 2, size=row.shape, dtype=np.int8)
        up, down = r > 0, r < 0
        row[up] = np.nextafter(row[up], np.inf)
        row[down] = np.nextafter(row[down], -np.inf)
    return a


def jitter_state(Q, G, L, seed=8965):
    return jitter(Q, seed), jitter(G, seed + 1), jitter(L, seed + 2)


def rms(a):
    return float(np.sqrt(np.mean(np.square(a)))) if np.size(a) else 0.0


def group_rms(A):
    """rms of each variable group of an array whose first axis is the conserved variable."""
    A = as_np(A)
    return {g: rms(A[v]) for g, v in GROUPS.items()}


def spread(ref, alt):
    """Per variable group: rms of the reference and of the second evaluation's difference."""
    ref, alt = as_np(ref), as_np(alt)
    return {g: {"ref": rms(ref[v]), "diff": rms(alt[v] - ref[v])} for g, v in GROUPS.items()}


def bar(sp, g):
    return max(TOL * sp[g]["ref"], FACTOR * sp[g]["diff"])


def assert_spread_parity(gpu, ref, sp, what):
    """GPU array against the oracle's, per variable group, at the measured bar of `sp`
    (a dict of spread())."""
    gpu, ref = as_np(gpu), as_np(ref)
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    for g, v in GROUPS.items():
        err = rms(gpu[v] - ref[v])
        b = bar(sp, g)
        assert err <= b, (what, g, err, b, sp[g])


def oracle_run_pair(dims, nodes, prm, Q, G, L, nsteps, dt=0.0):
    """The oracle's run (IEEE build, given inputs) and its spread: the FMA build on jittered
    inputs.  Returns ((Q, G, L), {"Q": spread, "G": spread, "L": spread}, last dt)."""
    nodes = as_np(nodes)
    a = tuple(as_np(x) for x in (Q, G, L))
    st, Qo, Go, Lo, dto, _ = O.run(dims, nodes, prm, *a, nsteps, dt=dt)
    assert st == 0, st
    st, Qa, Ga, La, _, _ = O.run(dims, nodes, prm, *jitter_state(*a), nsteps, dt=dt, variant="fma")
    assert st == 0, st
    return (Qo, Go, Lo), {"Q": spread(Qo, Qa), "G": spread(Go, Ga), "L": spread(Lo, La)}, dto


def stage1_cells_pair(dims, nodes, prm, dt, Q, G, L, cells):
    """Stage 1 of the listed cells by the oracle and its spread (as oracle_run_pair); arrays
    with the variable first: Q [5, n], G [5, 3, n], L [5, 12, n]."""
    nodes = as_np(nodes)
    a = tuple(as_np(x) for x in (Q, G, L))
    st, oq, og, ol = O.stage1_cells(dims, nodes, prm, dt, *a, cells)
    assert st == 0, st
    st, aq, ag, al = O.stage1_cells(dims, nodes, prm, dt, *jitter_state(*a), cells, variant="fma")
    assert st == 0, st
    tr = lambda q, g, l: (q.T, g.transpose(1, 2, 0), l.transpose(1, 2, 0))
    ref, alt = tr(oq, og, ol), tr(aq, ag, al)
    return ref, {k: spread(x, y) for k, x, y in zip("QGL", ref, alt)}


def assert_rel(gpu, ref, what, tol=TOL):
    gpu, ref = as_np(gpu), as_np(ref)
    nr = np.linalg.norm(ref)
    err = np.linalg.norm(gpu - ref) / (nr if nr > 0 else 1.0)
    assert err <= tol, (what, err)
