"""CPU checks of the seeded input generators (shared by the oracle and the GPU tests; they hold
none of the method's arithmetic)."""
import math

import numpy as np
import torch

from paper_2508_08965_amd import workloads as W


def test_multiblock_sizes_are_seeded_and_in_range():
    a, b = W.multiblock_dims(), W.multiblock_dims()
    assert a == b and len(a) == 24
    for nx, ny, nz in a:
        assert 32 <= nx <= 160 and 32 <= ny <= 96 and 32 <= nz <= 64
    assert W.multiblock_dims(seed=1) != a


def test_perturbed_mesh_is_periodic_and_positive():
    n = (6, 5, 4)
    nodes = W.perturbed_nodes(n, amp=0.05).numpy()
    per = 2 * math.pi
    np.testing.assert_allclose(nodes[:, :, -1, 0], nodes[:, :, 0, 0] + per, atol=1e-13)
    np.testing.assert_allclose(nodes[:, -1, :, 1], nodes[:, 0, :, 1] + per, atol=1e-13)
    np.testing.assert_allclose(nodes[-1, :, :, 2], nodes[0, :, :, 2] + per, atol=1e-13)
    assert np.all(np.diff(nodes[..., 0], axis=2) > 0)


def test_isotropic_turbulence_turbulent_mach_number_and_seed():
    n = 16
    f = W.isotropic_turbulence(n, k0=4.0, Mt=0.5, seed=8965)
    h = 2 * math.pi / n
    ax = torch.arange(n, dtype=torch.float64) * h
    x, y, z = torch.meshgrid(ax, ax, ax, indexing="ij")
    rho, u, v, w, p = f(x, y, z)
    # at the grid points the field is the generated one: rms speed / c = Mt with c = 1
    c = math.sqrt(1.4 * float(p.mean()) / float(rho.mean()))
    mt = math.sqrt(float((u ** 2 + v ** 2 + w ** 2).mean())) / c
    assert abs(mt - 0.5) < 1e-12 and abs(c - 1.0) < 1e-12
    g = W.isotropic_turbulence(n, k0=4.0, Mt=0.5, seed=8966)
    assert not torch.equal(g(x, y, z)[1], u)


def test_initial_state_of_uniform_flow_is_uniform():
    n = (5, 4, 3)
    Q, G, L = W.initial_state(W.perturbed_nodes(n, amp=0.05), W.uniform(), 1.4)
    assert float((Q - Q[:, :1]).abs().max()) < 1e-12 * float(Q.abs().max())
    assert float(G.abs().max()) < 1e-9 and float(L.abs().max()) < 1e-9
