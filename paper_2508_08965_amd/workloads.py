"""Seeded synthetic inputs: meshes and initial states.

This module holds none of the scheme's arithmetic.  It builds node arrays and
initial conserved states (cell averages, cell-averaged gradients and Gauss-point
differences) of closed-form or seeded random fields by plain quadrature, so that
the GPU library and the CPU oracle receive identical inputs.

Layouts match the library's C-ABI: nodes[(nz+1),(ny+1),(nx+1),3] (x fastest),
Q[5,N], G[5,3,N], L[5,12,N] with N = nx*ny*nz and cell c = i + nx*(j + ny*k).

Workloads (shapes and distributions of the paper's tests):
  * density_wave   -- advection of rho = 1 + 0.2 sin(pi(x+y[+z])), U=V(=W)=1, p=1
                      (accuracy test of Sec. 5.1; 2D variant as one periodic layer)
  * taylor_green   -- TGV initial field of Sec. 5.2 (Re 1600, Ma 0.1)
  * double_sod     -- periodic double shock tube (1D Riemann check)
  * uniform        -- free stream
  * isotropic_turbulence -- random-phase solenoidal field with E(k) ~ k^4 exp(-2k^2/k0^2)
"""
from __future__ import annotations

import math

import numpy as np
import torch

F64 = torch.float64

# 4-point Gauss-Legendre on [-1/2, 1/2]
_GL4_X = [-0.4305681557970263, -0.1699905217924281, 0.1699905217924281, 0.4305681557970263]
_GL4_W = [0.17392742256872692, 0.32607257743127307, 0.32607257743127307, 0.17392742256872692]
# Gauss points of the state's line differences: +-1/(2 sqrt 3) on the unit face
_GQ = 0.5 / math.sqrt(3.0)


# ----------------------------------------------------------------------------- meshes
def cartesian_nodes(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), device="cpu"):
    """Uniform nodes of an nx x ny x nz box; returns tensor [(nz+1),(ny+1),(nx+1),3]."""
    nx, ny, nz = n
    xs = [torch.linspace(lo[q], hi[q], n[q] + 1, dtype=F64, device=device) for q in range(3)]
    z, y, x = torch.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return torch.stack([x, y, z], dim=-1).contiguous()


def perturbed_nodes(n, amp=0.05, period=2.0 * math.pi, device="cpu"):
    """Periodic box [0, period]^3 with x = xi + amp sin(xi) sin(eta) sin(zeta) on every axis
    (the perturbed curvilinear TGV mesh); angles are 2 pi xi / period."""
    nx, ny, nz = n
    xs = [torch.arange(n[q] + 1, dtype=F64, device=device) * (period / n[q]) for q in range(3)]
    z, y, x = torch.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    k = 2.0 * math.pi / period
    s = torch.sin(k * x) * torch.sin(k * y) * torch.sin(k * z) * (amp * period / (2.0 * math.pi))
    return torch.stack([x + s, y + s, z + s], dim=-1).contiguous()


def skewed_nodes(n, period=1.0, shear=(0.3, 0.2, 0.1), device="cpu"):
    """Periodic affine (parallelepiped) mesh: x = xi + shear_0 eta, y = eta + shear_1 zeta,
    z = zeta + shear_2 xi, with lattice periods consistent with periodicity."""
    xs = [torch.arange(n[q] + 1, dtype=F64, device=device) * (period / n[q]) for q in range(3)]
    z, y, x = torch.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return torch.stack([x + shear[0] * y, y + shear[1] * z, z + shear[2] * x], dim=-1).contiguous()


def stretched_nodes(n, half=(math.pi, math.pi, math.pi), cells_per_half=None, amp=(0.1, 0.07, 0.05),
                    device="cpu"):
    """Stretched Cartesian nodes: along axis q, x_i = half_q (s + amp_q sin(pi s)) with
    s = i / cells_per_half_q, i = 0..n_q.  The map is odd about s = 0 and s = 1, so with
    n = cells_per_half the block [0, half] has mirror-symmetric spacing about its sides, and
    with n = 2 cells_per_half it is the periodic box [0, 2 half] whose first octant carries the
    same nodes (walls versus the doubled periodic domain)."""
    m = cells_per_half or n
    xs = []
    for q in range(3):
        s = torch.arange(n[q] + 1, dtype=F64, device=device) / m[q]
        xs.append(half[q] * (s + amp[q] * torch.sin(math.pi * s)))
    z, y, x = torch.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return torch.stack([x, y, z], dim=-1).contiguous()


def wall_perturbed_nodes(n, length=math.pi, amp=0.05, device="cpu"):
    """Curvilinear box [0, length]^3 whose six sides stay planes normal to the axes:
    x_d = xi_d + amp (length/pi) sin(pi xi_d/length) prod_{e != d} cos(2 pi xi_e/length).
    The tangential node coordinates agree on opposite sides (cos 0 = cos 2 pi)."""
    xs = [torch.arange(n[q] + 1, dtype=F64, device=device) * (length / n[q]) for q in range(3)]
    z, y, x = torch.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    a, k = amp * length / math.pi, math.pi / length
    cx, cy, cz = torch.cos(2 * k * x), torch.cos(2 * k * y), torch.cos(2 * k * z)
    dx = a * torch.sin(k * x) * cy * cz
    dy = a * torch.sin(k * y) * cx * cz
    dz = a * torch.sin(k * z) * cx * cy
    return torch.stack([x + dx, y + dy, z + dz], dim=-1).contiguous()


def shear_wave(U=0.05, H=1.0, mode="sin", rho=1.0, p=1.0 / 1.4):
    """Parallel shear flow u(y) = U sin(pi y/H) (no-slip walls at y = 0, H) or U cos(pi y/H)
    (symmetry planes), v = w = 0, uniform rho and p.  For a constant viscosity its
    incompressible decay is u(y) exp(-nu pi^2 t/H^2)."""

    def f(x, y, z):
        arg = math.pi * y / H
        u = U * (torch.sin(arg) if mode == "sin" else torch.cos(arg))
        zero = torch.zeros_like(x)
        return rho + zero, u, zero, zero, p + zero
    return f


# ----------------------------------------------------------------------------- trilinear cells
def _corners(nodes):
    c = {}
    for ck in (0, 1):
        for cj in (0, 1):
            for ci in (0, 1):
                c[(ci, cj, ck)] = nodes[ck:nodes.shape[0] - 1 + ck, cj:nodes.shape[1] - 1 + cj,
                                        ci:nodes.shape[2] - 1 + ci]
    return c


def _map(corners, xi):
    """Trilinear map on [-1/2,1/2]^3 at reference point xi: X [nz,ny,nx,3], J [..,3,3] (dX_i/dxi_j)."""
    X = 0.0
    J = [0.0, 0.0, 0.0]
    for (ci, cj, ck), p in corners.items():
        f = [0.5 + xi[0] if ci else 0.5 - xi[0], 0.5 + xi[1] if cj else 0.5 - xi[1],
             0.5 + xi[2] if ck else 0.5 - xi[2]]
        d = [1.0 if ci else -1.0, 1.0 if cj else -1.0, 1.0 if ck else -1.0]
        X = X + p * (f[0] * f[1] * f[2])
        J[0] = J[0] + p * (d[0] * f[1] * f[2])
        J[1] = J[1] + p * (f[0] * d[1] * f[2])
        J[2] = J[2] + p * (f[0] * f[1] * d[2])
    return X, J


def _det(J):
    a, b, c = J
    return (a[..., 0] * (b[..., 1] * c[..., 2] - b[..., 2] * c[..., 1])
            - b[..., 0] * (a[..., 1] * c[..., 2] - a[..., 2] * c[..., 1])
            + c[..., 0] * (a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1]))


def _cross(a, b):
    return torch.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                        a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                        a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], dim=-1)


def conserved(prim, gamma):
    """(rho, U, V, W, p) tensors -> stacked conserved variables [5, ...]."""
    rho, u, v, w, p = prim
    return torch.stack([rho, rho * u, rho * v, rho * w,
                        p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])


def initial_state(nodes, prim_fn, gamma=1.4):
    """Cell averages Q, cell-averaged gradients G (surface integral) and Gauss-point differences L
    of the field prim_fn(x, y, z) -> (rho, U, V, W, p) on the mesh given by nodes.
    Returns numpy-free torch tensors Q[5,N], G[5,3,N], L[5,12,N] on the nodes' device."""
    nodes = nodes.to(F64)
    nz, ny, nx = nodes.shape[0] - 1, nodes.shape[1] - 1, nodes.shape[2] - 1
    N = nx * ny * nz
    cr = _corners(nodes)

    def field(X):
        return conserved(prim_fn(X[..., 0], X[..., 1], X[..., 2]), gamma)

    vol = 0.0
    Qs = 0.0
    for a, wa in zip(_GL4_X, _GL4_W):
        for b, wb in zip(_GL4_X, _GL4_W):
            for c, wc in zip(_GL4_X, _GL4_W):
                X, J = _map(cr, (a, b, c))
                dj = _det(J) * (wa * wb * wc)
                vol = vol + dj
                Qs = Qs + field(X) * dj
    Q = Qs / vol
    # surface integral of Q n over the six bilinear faces (4x4 Gauss per face)
    Gs = torch.zeros((5, 3, nz, ny, nx), dtype=F64, device=nodes.device)
    for q in range(3):
        q1, q2 = (q + 1) % 3, (q + 2) % 3
        for side, sgn in ((-0.5, -1.0), (0.5, 1.0)):
            for a, wa in zip(_GL4_X, _GL4_W):
                for b, wb in zip(_GL4_X, _GL4_W):
                    xi = [0.0, 0.0, 0.0]
                    xi[q] = side
                    xi[q1] = a
                    xi[q2] = b
                    X, J = _map(cr, xi)
                    S = _cross(J[q1], J[q2]) * (sgn * wa * wb)
                    f = field(X)
                    Gs = Gs + f[:, None] * S.permute(3, 0, 1, 2)[None]
    G = Gs / vol
    # Gauss-point differences along the 12 lines (ascending tangential axes)
    Ls = []
    for q in range(3):
        ta, tb = [t for t in range(3) if t != q]
        for k in range(4):
            xm = [0.0, 0.0, 0.0]
            xm[ta] = (2 * (k & 1) - 1) * _GQ
            xm[tb] = (2 * (k >> 1) - 1) * _GQ
            xp = list(xm)
            xm[q], xp[q] = -0.5, 0.5
            Xm, _ = _map(cr, xm)
            Xp, _ = _map(cr, xp)
            Ls.append(field(Xp) - field(Xm))
    L = torch.stack(Ls, dim=1)
    return (Q.reshape(5, N).contiguous(), G.reshape(5, 3, N).contiguous(),
            L.reshape(5, 12, N).contiguous())


def exact_cell_average(nodes, fn):
    """Cell average of a scalar field fn(x, y, z) by 4^3 Gauss on each trilinear cell: [N]."""
    nodes = nodes.to(F64)
    cr = _corners(nodes)
    vol = 0.0
    s = 0.0
    for a, wa in zip(_GL4_X, _GL4_W):
        for b, wb in zip(_GL4_X, _GL4_W):
            for c, wc in zip(_GL4_X, _GL4_W):
                X, J = _map(cr, (a, b, c))
                dj = _det(J) * (wa * wb * wc)
                vol = vol + dj
                s = s + fn(X[..., 0], X[..., 1], X[..., 2]) * dj
    return (s / vol).reshape(-1)


# ----------------------------------------------------------------------------- fields
def density_wave(dim=3, amp=0.2):
    """rho = 1 + amp sin(pi(x+y[+z])), unit velocity on the active axes, p = 1."""
    def f(x, y, z):
        s = x + y + (z if dim == 3 else 0.0)
        rho = 1.0 + amp * torch.sin(math.pi * s)
        one = torch.ones_like(x)
        return rho, one, one, (one if dim == 3 else torch.zeros_like(x)), one
    return f


def density_wave_exact(t, dim=3, amp=0.2):
    def f(x, y, z):
        s = x + y + (z if dim == 3 else 0.0)
        return 1.0 + amp * torch.sin(math.pi * (s - dim * t))
    return f


def taylor_green(Ma=0.1, gamma=1.4, U0=1.0, rho0=1.0, L=1.0):
    """Taylor-Green vortex initial field of Sec. 5.2: p0 = rho0 U0^2 / (gamma Ma^2)."""
    p0 = rho0 * U0 * U0 / (gamma * Ma * Ma)

    def f(x, y, z):
        u = U0 * torch.sin(x / L) * torch.cos(y / L) * torch.cos(z / L)
        v = -U0 * torch.cos(x / L) * torch.sin(y / L) * torch.cos(z / L)
        w = torch.zeros_like(x)
        fac = 1.0 + gamma * Ma * Ma / 16.0 * (torch.cos(2 * x / L) + torch.cos(2 * y / L)) * (torch.cos(2 * z / L) + 2.0)
        return rho0 * fac, u, v, w, p0 * fac
    return f


def uniform(rho=1.0, u=0.5, v=0.3, w=0.2, p=1.0 / 0.014):
    def f(x, y, z):
        one = torch.ones_like(x)
        return rho * one, u * one, v * one, w * one, p * one
    return f


def double_sod():
    """Periodic double shock tube on [0,1): (1, 0, 1) on [0.25, 0.75), (0.125, 0, 0.1) elsewhere."""
    def f(x, y, z):
        inside = (x >= 0.25) & (x < 0.75)
        rho = torch.where(inside, torch.ones_like(x), 0.125 * torch.ones_like(x))
        p = torch.where(inside, torch.ones_like(x), 0.1 * torch.ones_like(x))
        zero = torch.zeros_like(x)
        return rho, zero, zero, zero, p
    return f


def isotropic_turbulence(n, k0=4.0, Mt=0.5, gamma=1.4, seed=8965, period=2.0 * math.pi):
    """Random-phase solenoidal velocity with E(k) ~ k^4 exp(-2 k^2/k0^2) on an n^3 periodic grid,
    scaled so that sqrt(<U.U>)/c = Mt with rho = 1, p = 1/gamma (c = 1).  Returns a field function
    that samples the grid field by trilinear interpolation (periodic)."""
    g = np.random.default_rng(seed)
    kk = np.fft.fftfreq(n, d=1.0 / n)
    kx, ky, kz = np.meshgrid(kk, kk, kk, indexing="ij")
    kmag = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    kmag[0, 0, 0] = 1.0
    amp = np.sqrt(kmag ** 4 * np.exp(-2.0 * kmag ** 2 / k0 ** 2) / (4.0 * math.pi * kmag ** 2))
    amp[0, 0, 0] = 0.0
    vel = []
    for _ in range(3):
        ph = g.uniform(0, 2 * math.pi, size=kmag.shape)
        vel.append(amp * np.exp(1j * ph))
    vx, vy, vz = vel
    kd = (kx * vx + ky * vy + kz * vz) / kmag ** 2
    vx, vy, vz = vx - kx * kd, vy - ky * kd, vz - kz * kd
    u = [np.real(np.fft.ifftn(c)) for c in (vx, vy, vz)]
    urms = math.sqrt(np.mean(u[0] ** 2 + u[1] ** 2 + u[2] ** 2))
    scale = Mt / urms
    grid = [torch.from_numpy(np.ascontiguousarray(c * scale)) for c in u]
    p_amb = 1.0 / gamma
    h = period / n

    def f(x, y, z):
        dev = x.device
        gx = [t.to(dev) for t in grid]
        fx, fy, fz = x / h, y / h, z / h
        ix, iy, iz = torch.floor(fx), torch.floor(fy), torch.floor(fz)
        tx, ty, tz = fx - ix, fy - iy, fz - iz
        ix, iy, iz = ix.long() % n, iy.long() % n, iz.long() % n
        out = []
        for comp in gx:
            acc = 0.0
            for dx in (0, 1):
                for dy in (0, 1):
                    for dz in (0, 1):
                        wgt = (tx if dx else 1 - tx) * (ty if dy else 1 - ty) * (tz if dz else 1 - tz)
                        acc = acc + wgt * comp[(ix + dx) % n, (iy + dy) % n, (iz + dz) % n]
            out.append(acc)
        one = torch.ones_like(x)
        return one, out[0], out[1], out[2], p_amb * one
    return f


def multiblock_dims(nblocks=24, seed=8965):
    """Uneven block sizes of the multi-block batching workload: nx in [32, 160], ny in [32, 96],
    nz in [32, 64], drawn per block from one seeded generator."""
    g = np.random.default_rng(seed)
    dims = []
    for _ in range(nblocks):
        nx = int(g.integers(32, 161))
        ny = int(g.integers(32, 97))
        nz = int(g.integers(32, 65))
        dims.append((nx, ny, nz))
    return dims
