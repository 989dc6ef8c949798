"""Whole-run GPU parity at the sizes of the Taylor-Green configurations, through the C ABI.

* 128^3 curvilinear Taylor-Green vortex (Re 1600, Ma 0.1, Pr 0.72, Sutherland), 20 S2O4 steps
  at CFL 0.5: the parity configuration behind the 256^3 benchmark.  The oracle takes minutes
  here, so the GPU and the oracle advance side by side in chunks of 5 steps and each chunk is
  a test of its own (results after 5, 10, 15 and 20 steps); every chunk compares the whole
  state element by element.
* 64^3, same flow, 50 steps: the chain that lets the GPU FP64 run serve as the FP64 reference
  of the 256^3 reduced-precision errors.

Q is held to 1e-12 relative L2; G and L to twice the oracle's own rounding spread
(tests/parity_bar.py), taken from tests/golden/oracle_spread.json (written by
tests/golden/make_oracle_spread.py, which runs only the oracle; these runs are too long to
repeat here).  A stored spread applies only to the oracle result it was measured on: the
stored rms of the oracle's result must equal the live one's.  Progress lines go to the
terminal after every chunk.
"""
import json
import os

import pytest
import torch

import parity_bar as PB
from oracle import oracle as O
from paper_2508_08965_amd import workloads as W

pytestmark = pytest.mark.gpu

GAM = 1.4
HERE = os.path.dirname(os.path.abspath(__file__))
SPREAD = os.path.join(HERE, "golden", "oracle_spread.json")


def K():
    from paper_2508_08965_amd import cgks
    return cgks


def dev():
    return torch.device("cuda:0")


def tgv_kw():
    p0 = 1.0 / (GAM * 0.1 * 0.1)
    return dict(viscous=1, visc_law=1, mu0=1.0 / 1600.0, T_ref=p0, S_suth=p0 * 110.4 / 288.15, Pr=0.72,
                prandtl_fix=1)


def stored_spread(case, step, oracle_state):
    """The stored spread of `case` at `step`, after checking that it was measured on this
    oracle result (per variable group, the rms of Q, G and L to 1e-12)."""
    sp = json.load(open(SPREAD))["cases"][case]["checkpoints"][str(step)]
    for kind, arr in zip("QGL", oracle_state):
        live = PB.group_rms(arr)
        for g in PB.GROUPS:
            assert live[g] == pytest.approx(sp[kind][g]["ref"], rel=1e-12), \
                ("oracle result differs from the stored one: rerun tests/golden/make_oracle_spread.py", kind, g)
    return sp


def say(capsys, msg):
    with capsys.disabled():
        print(msg, flush=True)


class SideBySide:
    """GPU context and oracle state of one workload, advanced together."""

    def __init__(self, n):
        self.n = n
        nodes = W.perturbed_nodes(n, amp=0.05)
        Q, G, L = W.initial_state(nodes, W.taylor_green(Ma=0.1), GAM)
        self.nodes = nodes.numpy()
        self.oracle = (Q.numpy(), G.numpy(), L.numpy())
        self.ctx = K().Context([n], [nodes], K().default_params(**tgv_kw()))
        self.gpu = [t.to(dev()) for t in (Q, G, L)]
        self.dt = torch.zeros(1, dtype=torch.float64, device=dev())
        self.steps = 0
        self.prm = O.params(**tgv_kw())

    def advance(self, to, capsys, chunk=5):
        while self.steps < to:
            k = min(chunk, to - self.steps)
            for _ in range(k):
                K().cgks_step(self.ctx, *self.gpu, self.dt, use_cfl=True)
            torch.cuda.synchronize()
            assert K().cgks_check(self.ctx) == (0, 0)
            st, Qo, Go, Lo, _, _ = O.run(self.n, self.nodes, self.prm, *self.oracle, k)
            assert st == 0
            self.oracle = (Qo, Go, Lo)
            self.steps += k
            say(capsys, f"  {self.n[0]}^3 Taylor-Green: GPU and oracle at step {self.steps}")

    def close(self):
        self.ctx.close()


@pytest.fixture(scope="module")
def c1():
    box = {}
    yield box
    if "run" in box:
        box["run"].close()


@pytest.mark.parametrize("step", [5, 10, 15, 20])
def test_tgv128_whole_state_parity(c1, step, capsys):
    if "run" not in c1:
        c1["run"] = SideBySide((128, 128, 128))
    run = c1["run"]
    run.advance(step, capsys)
    sp = stored_spread("tgv_curvilinear_128", step, run.oracle)
    got = [t.cpu().numpy() for t in run.gpu]
    PB.assert_rel(got[0], run.oracle[0], "Q")
    PB.assert_spread_parity(got[1], run.oracle[1], sp["G"], "G")
    PB.assert_spread_parity(got[2], run.oracle[2], sp["L"], "L")


def test_tgv64_fifty_steps_whole_state_parity(capsys):
    run = SideBySide((64, 64, 64))
    try:
        run.advance(50, capsys, chunk=25)
        sp = stored_spread("tgv_curvilinear_64", 50, run.oracle)
        got = [t.cpu().numpy() for t in run.gpu]
        PB.assert_rel(got[0], run.oracle[0], "Q")
        PB.assert_spread_parity(got[1], run.oracle[1], sp["G"], "G")
        PB.assert_spread_parity(got[2], run.oracle[2], sp["L"], "L")
    finally:
        run.close()
