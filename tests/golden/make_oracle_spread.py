"""Writes tests/golden/oracle_spread.json: the oracle's own FP64 rounding spread on the
whole-run parity workloads whose oracle runs are too long to repeat inside the GPU tests.

For each workload the oracle (IEEE build) runs from the seeded initial state, and a second
evaluation runs the FMA-contracted build from the same state with every value jittered by at
most one unit in the last place (tests/parity_bar.py).  The file stores, per variable group of
Q, G and L, the rms of the oracle's result and of the second evaluation's difference, at each
checkpoint the GPU tests compare (a test uses a stored spread only where the stored rms of the
oracle's result equals the live one's); the digest of the oracle source is recorded for
reference.  Calls only oracle/ and the shared input generators.

Usage: python tests/golden/make_oracle_spread.py [case ...]
"""
import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import oracle as O  # noqa: E402
from paper_2508_08965_amd import workloads as W  # noqa: E402
import parity_bar as PB  # noqa: E402

GAM = 1.4
OUT = os.path.join(HERE, "oracle_spread.json")


def oracle_digest():
    with open(O.SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def tgv_params():
    """Taylor-Green vortex: Re 1600, Ma 0.1, Pr 0.72, Sutherland viscosity (Sec. 5)."""
    p0 = 1.0 / (GAM * 0.1 * 0.1)
    return O.params(viscous=1, visc_law=1, mu0=1.0 / 1600.0, T_ref=p0, S_suth=p0 * 110.4 / 288.15, Pr=0.72,
                    prandtl_fix=1)


# name: (cells per axis, checkpoints in steps)
CASES = {
    "tgv_curvilinear_20x18x16": ((20, 18, 16), [6]),
    "tgv_curvilinear_64": ((64, 64, 64), [50]),
    "tgv_curvilinear_128": ((128, 128, 128), [5, 10, 15, 20]),
}


def run_case(dims):
    nodes = W.perturbed_nodes(dims, amp=0.05).numpy()
    Q, G, L = W.initial_state(W.perturbed_nodes(dims, amp=0.05), W.taylor_green(Ma=0.1), GAM)
    a = (Q.numpy(), G.numpy(), L.numpy())
    b = PB.jitter_state(*a)
    return nodes, a, b


def main(names):
    rec = json.load(open(OUT)) if os.path.exists(OUT) else {}
    rec["oracle_sha256"] = oracle_digest()
    rec.setdefault("cases", {})
    prm = tgv_params()
    for name in names:
        dims, checkpoints = CASES[name]
        nodes, a, b = run_case(dims)
        done, out, t0 = 0, {}, time.time()
        for cp in checkpoints:
            k = cp - done
            st, *ra = O.run(dims, nodes, prm, *a, k)[:4]
            assert st == 0, (name, st)
            st, *rb = O.run(dims, nodes, prm, *b, k, variant="fma")[:4]
            assert st == 0, (name, st)
            a, b, done = tuple(ra), tuple(rb), cp
            out[str(cp)] = {n: PB.spread(x, y) for n, x, y in zip("QGL", a, b)}
            print(f"{name}: step {cp} ({time.time() - t0:.0f} s)", flush=True)
        rec["cases"][name] = {"dims": list(dims), "checkpoints": out}
        rec["oracle_sha256"] = oracle_digest()
        with open(OUT, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
