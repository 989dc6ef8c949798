// HIP kernels of the CGKS-5 stage path for gfx950 (FP64 path).
//
//   k_metrics   : per-cell geometry (Sec. 4 J0 and (J0^T)^-1; Appendix trilinear volume;
//                 2x2 Gauss points of the bilinear faces, Sec. 2)
//   k_dt_*      : CFL time step, min over cells (Sec. 5)
//   k_recon     : compact reconstruction on the standard cell + GENO blend (Sec. 3.3, 4)
//   (the gas-kinetic flux at the face Gauss points is in cgks_flux.hip)
//   k_update    : face -> cell accumulation and S2O4 stage update (Sec. 3.1, temporal section)
//
// Data layout (SoA, stride Ntot = cells of all blocks, x fastest inside a block):
//   gp  [q][side][k][v*4 + c][Gtot]   reconstructed value (c = 0) and physical gradient
//                                     (c = 1..3) at Gauss point k of face q of the face
//                                     record owned by the minus-side cell; side 0 = values
//                                     of the minus-side (left) cell, side 1 = plus-side cell;
//                                     cells at gp_at(), rows padded to 16 cells.
//   fo  [q][k][30][Ntot]              F^n (5), F_t^n (5), Q^l, dQ^l/dt, Q^r, dQ^r/dt (20)
#include <hip/hip_runtime.h>

#include "cgks_device.h"

namespace cgks {

// ------------------------------------------------------------------------------------------
// small device helpers
// ------------------------------------------------------------------------------------------
struct Idx3 {
    int i, j, k;
};

__device__ inline Idx3 unflatten(const BlockView &b, long cl) {
    Idx3 r;
    r.i = (int)(cl % b.nx);
    long t = cl / b.nx;
    r.j = (int)(t % b.ny);
    r.k = (int)(t / b.ny);
    return r;
}

__device__ inline long cell_at(const BlockView &b, int i, int j, int k) {
    i = (i < 0) ? i + b.nx : (i >= b.nx ? i - b.nx : i);
    j = (j < 0) ? j + b.ny : (j >= b.ny ? j - b.ny : j);
    k = (k < 0) ? k + b.nz : (k >= b.nz ? k - b.nz : k);
    return b.off + (long)i + (long)b.nx * ((long)j + (long)b.ny * k);
}

__device__ inline const double *node_ptr(const double *nodes, const BlockView &b, int i, int j, int k) {
    return nodes + 3 * ((long)i + (long)(b.nx + 1) * ((long)j + (long)(b.ny + 1) * k));
}

// ------------------------------------------------------------------------------------------
// metrics
// ------------------------------------------------------------------------------------------
// Bilinear face with corners P00, P10, P01, P11 over (s,t) in [-1/2,1/2]^2: area vector
// dX/ds x dX/dt at (s,t).
__device__ inline void face_area_vec(const double *P00, const double *P10, const double *P01,
                                     const double *P11, double s, double t, double out[3]) {
    double ds[3], dt[3];
    for (int r = 0; r < 3; ++r) {
        ds[r] = (0.5 - t) * (P10[r] - P00[r]) + (0.5 + t) * (P11[r] - P01[r]);
        dt[r] = (0.5 - s) * (P01[r] - P00[r]) + (0.5 + s) * (P11[r] - P10[r]);
    }
    out[0] = ds[1] * dt[2] - ds[2] * dt[1];
    out[1] = ds[2] * dt[0] - ds[0] * dt[2];
    out[2] = ds[0] * dt[1] - ds[1] * dt[0];
}

__global__ void __launch_bounds__(256) k_metrics(BlockView b, const double *__restrict__ nodes, Metrics M,
                                                 long Ntot, int *__restrict__ bad) {
    long cl = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cl >= b.N) return;
    Idx3 id = unflatten(b, cl);
    long c = b.off + cl;
    const double *P[8];
    for (int t = 0; t < 8; ++t) P[t] = node_ptr(nodes, b, id.i + (t & 1), id.j + ((t >> 1) & 1), id.k + (t >> 2));
    // volume: 2x2x2 Gauss of det dX/dxi (exact for a trilinear map)
    const double gq = 0.28867513459481288225;
    double vol = 0.0;
    for (int a = 0; a < 8; ++a) {
        double xi[3] = {(a & 1) ? gq : -gq, ((a >> 1) & 1) ? gq : -gq, (a >> 2) ? gq : -gq};
        double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int t = 0; t < 8; ++t) {
            double s0 = (t & 1) ? 1.0 : -1.0, s1 = ((t >> 1) & 1) ? 1.0 : -1.0, s2 = (t >> 2) ? 1.0 : -1.0;
            double f0 = 0.5 + s0 * xi[0], f1 = 0.5 + s1 * xi[1], f2 = 0.5 + s2 * xi[2];
            for (int r = 0; r < 3; ++r) {
                J[r][0] += P[t][r] * s0 * f1 * f2;
                J[r][1] += P[t][r] * f0 * s1 * f2;
                J[r][2] += P[t][r] * f0 * f1 * s2;
            }
        }
        double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        vol += 0.125 * det;
    }
    M.vol[c] = vol;
    // J0 = [N2 - N1, N3 - N1, N4 - N1] with N1 = node (i,j,k)
    double J0[3][3];
    for (int r = 0; r < 3; ++r) {
        J0[r][0] = P[1][r] - P[0][r];
        J0[r][1] = P[2][r] - P[0][r];
        J0[r][2] = P[4][r] - P[0][r];
    }
    double det = J0[0][0] * (J0[1][1] * J0[2][2] - J0[1][2] * J0[2][1]) - J0[0][1] * (J0[1][0] * J0[2][2] - J0[1][2] * J0[2][0]) +
                 J0[0][2] * (J0[1][0] * J0[2][1] - J0[1][1] * J0[2][0]);
    if (!(vol > 0.0) || !(det > 0.0)) atomicOr(bad, 1);
    double inv = 1.0 / det;
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
            M.J0[(3 * r + q) * Ntot + c] = J0[r][q];
            // ((J0^T)^-1)[r][q] = cofactor(J0)[r][q] / det
            int r1 = (r + 1) % 3, r2 = (r + 2) % 3, q1 = (q + 1) % 3, q2 = (q + 2) % 3;
            M.JiT[(3 * r + q) * Ntot + c] = (J0[r1][q1] * J0[r2][q2] - J0[r1][q2] * J0[r2][q1]) * inv;
        }
    // faces: for each axis the plus face (owned) and the minus face (for the time step)
    const double gpt = 0.28867513459481288225;
    double hsum[3];
    for (int q = 0; q < 3; ++q) {
        int a = (q == 0) ? 1 : 0, bb = (q == 2) ? 1 : 2;  // ascending tangential axes
        double S[2][3] = {{0, 0, 0}, {0, 0, 0}};
        double area[2] = {0, 0};
        for (int side = 0; side < 2; ++side) {
            // corners of the face: index along q fixed, (a, b) in {0,1}^2
            const double *C[4];
            for (int t = 0; t < 4; ++t) {
                int o[3] = {0, 0, 0};
                o[q] = side;
                o[a] = t & 1;
                o[bb] = t >> 1;
                C[t] = node_ptr(nodes, b, id.i + o[0], id.j + o[1], id.k + o[2]);
            }
            for (int kk = 0; kk < 4; ++kk) {
                double s = (kk & 1) ? gpt : -gpt, t = (kk >> 1) ? gpt : -gpt;
                double av[3];
                face_area_vec(C[0], C[1], C[2], C[3], s, t, av);
                if (q == 1) { av[0] = -av[0]; av[1] = -av[1]; av[2] = -av[2]; }  // cyclic (zeta, xi)
                double nrm = sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
                double wds = 0.25 * nrm;
                if (side == 1) {
                    for (int r = 0; r < 3; ++r) M.fn[((q * 4 + kk) * 3 + r) * Ntot + c] = av[r] / nrm;
                    M.fw[(q * 4 + kk) * Ntot + c] = wds;
                }
                for (int r = 0; r < 3; ++r) S[side][r] += 0.25 * av[r];
            }
            area[side] = sqrt(S[side][0] * S[side][0] + S[side][1] * S[side][1] + S[side][2] * S[side][2]);
        }
        double nb[3] = {S[0][0] + S[1][0], S[0][1] + S[1][1], S[0][2] + S[1][2]};
        double nl = sqrt(nb[0] * nb[0] + nb[1] * nb[1] + nb[2] * nb[2]);
        for (int r = 0; r < 3; ++r) M.dtm[(q * 4 + r) * Ntot + c] = nb[r] / nl;
        hsum[q] = vol / (0.5 * (area[0] + area[1]));
        M.dtm[(q * 4 + 3) * Ntot + c] = 1.0 / hsum[q];
    }
}

// ------------------------------------------------------------------------------------------
// time step
// ------------------------------------------------------------------------------------------
__device__ inline double viscosity_dt(const DevParams &P, double T) {
    if (!P.visc_law) return P.mu0;
    double r = T / P.T_ref;
    return P.mu0 * r * sqrt(r) * (P.T_ref + P.S_suth) / (T + P.S_suth);
}

__device__ inline double block_min(double v) {
    __shared__ double red[16];
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = fmin(m, red[i]);
        red[0] = m;
    }
    __syncthreads();
    return red[0];
}

__global__ void __launch_bounds__(256) k_dt_partial(long off, long N, long Ntot, const double *__restrict__ Q,
                                                    const double *__restrict__ dtm, DevParams P,
                                                    double *__restrict__ part, int *__restrict__ flag) {
    double best = INFINITY;
    for (long cl = (long)blockIdx.x * blockDim.x + threadIdx.x; cl < N; cl += (long)gridDim.x * blockDim.x) {
        long c = off + cl;
        double rho = Q[c], ru = Q[Ntot + c], rv = Q[2 * Ntot + c], rw = Q[3 * Ntot + c], re = Q[4 * Ntot + c];
        double u = ru / rho, v = rv / rho, w = rw / rho;
        double p = (P.gamma - 1.0) * (re - 0.5 * rho * (u * u + v * v + w * w));
        if (!(rho > 0.0) || !(p > 0.0)) {
            atomicOr(flag, !(rho > 0.0) ? 1 : 2);
            continue;
        }
        double cs = sqrt(P.gamma * p / rho);
        double rate = 0.0, ihmax = 0.0;
        for (int q = 0; q < 3; ++q) {
            double nx = dtm[(q * 4) * Ntot + c], ny = dtm[(q * 4 + 1) * Ntot + c], nz = dtm[(q * 4 + 2) * Ntot + c];
            double ih = dtm[(q * 4 + 3) * Ntot + c];
            rate += (fabs(u * nx + v * ny + w * nz) + cs) * ih;
            ihmax = fmax(ihmax, ih);
        }
        double d = P.cfl / rate;
        if (P.viscous) {
            double nu = viscosity_dt(P, p / rho) / rho;
            d = fmin(d, P.cfl / (ihmax * ihmax * 3.0 * nu));
        }
        best = fmin(best, d);
    }
    best = block_min(best);
    if (threadIdx.x == 0) part[blockIdx.x] = best;
}

__global__ void __launch_bounds__(256) k_dt_final(const double *__restrict__ part, int n, double *__restrict__ dt) {
    double best = INFINITY;
    for (int i = threadIdx.x; i < n; i += blockDim.x) best = fmin(best, part[i]);
    best = block_min(best);
    if (threadIdx.x == 0) *dt = best;
}

// ------------------------------------------------------------------------------------------
// flow diagnostics of the Taylor-Green section (Sec. 5): volume sums of the kinetic energy and
// the enstrophy (midpoint rule over cells, cell-averaged gradients), total mass and energy,
// minima of rho and p.  Fixed partition of the cells over the workgroups and a fixed summation
// tree: the result does not depend on timing.
// ------------------------------------------------------------------------------------------
constexpr int kDiagVals = 7;  // volume, mass, kinetic energy, enstrophy, energy; min rho, min p

__global__ void __launch_bounds__(256) k_diag_partial(long Ntot, const double *__restrict__ Q,
                                                      const double *__restrict__ G, const double *__restrict__ vol,
                                                      DevParams P, double *__restrict__ part) {
    __shared__ double red[kDiagVals][256];
    double acc[kDiagVals] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, INFINITY};
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < Ntot; c += (long)gridDim.x * blockDim.x) {
        const double v = vol[c], rho = Q[c];
        double U[3], uu = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            U[i] = Q[(1 + i) * Ntot + c] / rho;
            uu += U[i] * U[i];
        }
        const double k = 0.5 * rho * uu, re = Q[4 * Ntot + c];
        const double p = (P.gamma - 1.0) * (re - k);
        const double mu = viscosity_dt(P, p / rho);
        // velocity gradient from the cell-averaged gradients of rho and rho U
        double dU[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) dU[i][j] = (G[(3 * (1 + i) + j) * Ntot + c] - U[i] * G[j * Ntot + c]) / rho;
        const double w0 = dU[2][1] - dU[1][2], w1 = dU[0][2] - dU[2][0], w2 = dU[1][0] - dU[0][1];
        acc[0] += v;
        acc[1] += rho * v;
        acc[2] += k * v;
        acc[3] += mu * (w0 * w0 + w1 * w1 + w2 * w2) * v;
        acc[4] += re * v;
        acc[5] = fmin(acc[5], rho);
        acc[6] = fmin(acc[6], p);
    }
#pragma unroll
    for (int i = 0; i < kDiagVals; ++i) red[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int i = 0; i < 5; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + h];
#pragma unroll
            for (int i = 5; i < kDiagVals; ++i) red[i][threadIdx.x] = fmin(red[i][threadIdx.x], red[i][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < kDiagVals) part[(long)blockIdx.x * kDiagVals + threadIdx.x] = red[threadIdx.x][0];
}

// Q-criterion of every cell: (|Omega|^2 - |S|^2) / 2 of the velocity gradient
// (grad(rho U) - U grad rho) / rho; one thread per cell.
__global__ void __launch_bounds__(256) k_qcrit(long Ntot, const double *__restrict__ Q, const double *__restrict__ G,
                                               double *__restrict__ out) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= Ntot) return;
    const double rho = Q[c];
    double U[3], dU[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) U[i] = Q[(1 + i) * Ntot + c] / rho;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) dU[i][j] = (G[(3 * (1 + i) + j) * Ntot + c] - U[i] * G[j * Ntot + c]) / rho;
    double s2 = 0.0, o2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double sij = 0.5 * (dU[i][j] + dU[j][i]), oij = 0.5 * (dU[i][j] - dU[j][i]);
            s2 += sij * sij;
            o2 += oij * oij;
        }
    out[c] = 0.5 * (o2 - s2);
}

hipError_t launch_qcriterion(long Ntot, const double *Q, const double *G, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_qcrit, dim3((unsigned)((Ntot + 255) / 256)), dim3(256), 0, s, Ntot, Q, G, out);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_diag_final(const double *__restrict__ part, int n, double *__restrict__ out) {
    __shared__ double red[kDiagVals][256];
    double acc[kDiagVals] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, INFINITY};
    for (int b = threadIdx.x; b < n; b += blockDim.x) {
#pragma unroll
        for (int i = 0; i < 5; ++i) acc[i] += part[(long)b * kDiagVals + i];
#pragma unroll
        for (int i = 5; i < kDiagVals; ++i) acc[i] = fmin(acc[i], part[(long)b * kDiagVals + i]);
    }
#pragma unroll
    for (int i = 0; i < kDiagVals; ++i) red[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int i = 0; i < 5; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + h];
#pragma unroll
            for (int i = 5; i < kDiagVals; ++i) red[i][threadIdx.x] = fmin(red[i][threadIdx.x], red[i][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double V = red[0][0], m = red[1][0];
        out[0] = red[2][0] / m;  // E_k = int rho U.U / 2 / (rho0 |Omega|), rho0 = m / V
        out[1] = red[3][0] / m;  // eps_S = int mu |curl U|^2 / (rho0 |Omega|)
        out[2] = m / V;
        out[3] = red[4][0] / V;
        out[4] = red[5][0];
        out[5] = red[6][0];
    }
}

// ------------------------------------------------------------------------------------------
// reconstruction + GENO blend: one thread per (cell, conserved variable)
// ------------------------------------------------------------------------------------------
// Coefficients of one cell and variable on the vector ALU (periodic blocks): the quartic's
// a = R b from the stencil data (eq. compact-big-ref), the path function chi and the weighted
// gradient bbar of the linear sub-polynomials (eq. weno-new, compact-sub-2).
__device__ inline void valu_coeffs(const BlockView &b, long Ntot, const double *__restrict__ Q,
                                   const double *__restrict__ G, const double *__restrict__ L, const Metrics &M,
                                   const DevConsts *__restrict__ K, const DevParams &P, long cl, int v, double &q0_out,
                                   double a[kNB], double &chi_out, double bbar[3]) {
    Idx3 id = unflatten(b, cl);
    const long c = b.off + cl;
    const double *Qv = Q + v * Ntot;
    const double *Gv = G + 3 * v * Ntot;
    const double *Lv = L + 12 * v * Ntot;

    double J0[3][3];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) J0[r][q] = M.J0[(3 * r + q) * Ntot + c];

    const double q0 = Qv[c];
    double bvec[kNR];
    long fnb[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        int o[3] = {0, 0, 0};
        o[m >> 1] = (m & 1) ? 1 : -1;
        fnb[m] = cell_at(b, id.i + o[0], id.j + o[1], id.k + o[2]);
        bvec[m] = Qv[fnb[m]] - q0;
        double g0 = Gv[fnb[m]], g1 = Gv[Ntot + fnb[m]], g2 = Gv[2 * Ntot + fnb[m]];
#pragma unroll
        for (int j = 0; j < 3; ++j) bvec[kRowFaceGrad + 3 * m + j] = J0[0][j] * g0 + J0[1][j] * g1 + J0[2][j] * g2;
    }
#pragma unroll
    for (int n = 0; n < 12; ++n) {
        const int pa = (n < 8) ? 0 : 1, pb = (n < 4) ? 1 : 2, pc = 3 - pa - pb;
        const int sa = (n & 1) ? 1 : -1, sb = (n & 2) ? 1 : -1;
        int o[3] = {0, 0, 0};
        o[pa] = sa;
        o[pb] = sb;
        long e = cell_at(b, id.i + o[0], id.j + o[1], id.k + o[2]);
        bvec[kRowEdgeAvg + n] = Qv[e] - q0;
        double g0 = Gv[e], g1 = Gv[Ntot + e], g2 = Gv[2 * Ntot + e];
        double gr[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) gr[j] = J0[0][j] * g0 + J0[1][j] * g1 + J0[2][j] * g2;
        bvec[kRowEdgeDir + 2 * n] = gr[pc];
        bvec[kRowEdgeDir + 2 * n + 1] = (sa * gr[pa] + sb * gr[pb]) * 0.70710678118654752440;
    }
    double lines[12];
#pragma unroll
    for (int s = 0; s < 12; ++s) {
        lines[s] = Lv[s * Ntot + c];
        bvec[kRowLine + s] = lines[s];
    }

    // low-order blend: linear polynomials of the six sub-stencils and their weights
    bbar[0] = bbar[1] = bbar[2] = 0.0;
    if (!P.linear) {
        double lm[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) lm[t] = 0.25 * (lines[4 * t] + lines[4 * t + 1] + lines[4 * t + 2] + lines[4 * t + 3]);
        double wsum = 0.0, wv[6], bm[6][3];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const int q = m >> 1;
#pragma unroll
            for (int t = 0; t < 3; ++t) bm[m][t] = (t == q) ? ((m & 1) ? bvec[m] : -bvec[m]) : lm[t];
            double is = bm[m][0] * bm[m][0] + bm[m][1] * bm[m][1] + bm[m][2] * bm[m][2] + P.geno_eps;
            double is2 = is * is;
            wv[m] = (1.0 / 6.0) / (is2 * is2 * is);
            wsum += wv[m];
        }
        double iw = 1.0 / wsum;
#pragma unroll
        for (int m = 0; m < 6; ++m)
#pragma unroll
            for (int t = 0; t < 3; ++t) bbar[t] += (wv[m] * iw) * bm[m][t];
    }

    // a = R b
#pragma unroll
    for (int r = 0; r < kNB; ++r) {
        double s = 0.0;
#pragma unroll
        for (int col = 0; col < kNR; ++col) s = fma(K->R[r][col], bvec[col], s);
        a[r] = s;
    }

    double chi = 1.0;
    if (!P.linear) {
        double isl = 0.0, ist = 0.0;
#pragma unroll
        for (int r = 0; r < kNB; ++r) {
            double tl = 0.0, tt = 0.0;
#pragma unroll
            for (int s = 0; s < kNB; ++s) {
                tl = fma(K->GL[r][s], a[s], tl);
                tt = fma(K->GT[r][s], a[s], tt);
            }
            isl = fma(a[r], tl, isl);
            ist = fma(a[r], tt, ist);
        }
        double ish = isl + ist;
        double rh = ist / (ish + P.geno_eps), rl = ist / (isl + P.geno_eps);
        double ah, al;
        if (P.geno_r == 2.0) {
            ah = 1.0 + rh * rh;
            al = 1.0 + rl * rl;
        } else {
            ah = 1.0 + pow(rh, P.geno_r);
            al = 1.0 + pow(rl, P.geno_r);
        }
        double alpha = 2.0 * ah / (ah + al);
        chi = tanh(P.geno_C * alpha) * P.inv_tanhC;
    }
    q0_out = q0;
    chi_out = chi;
}

__global__ void __launch_bounds__(256) k_recon(BlockView b, long Ntot, const double *__restrict__ Q,
                                               const double *__restrict__ G, const double *__restrict__ L,
                                               Metrics M, const DevConsts *__restrict__ K, DevParams P,
                                               double *__restrict__ gp) {
    long cl = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cl >= b.N) return;
    const int v = blockIdx.y;
    Idx3 id = unflatten(b, cl);
    const long c = b.off + cl;
    double q0, a[kNB], chi, bbar[3];
    valu_coeffs(b, Ntot, Q, G, L, M, K, P, cl, v, q0, a, chi, bbar);

    double JiT[3][3];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) JiT[r][q] = M.JiT[(3 * r + q) * Ntot + c];

    const double om = 1.0 - chi;
#pragma unroll 1
    for (int g = 0; g < kNGP; ++g) {
        double pv = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
        for (int r = 0; r < kNB; ++r) {
            pv = fma(K->E[g][0][r], a[r], pv);
            p1 = fma(K->E[g][1][r], a[r], p1);
            p2 = fma(K->E[g][2][r], a[r], p2);
            p3 = fma(K->E[g][3][r], a[r], p3);
        }
        const double *xg = K->xg[g];
        double low = bbar[0] * xg[0] + bbar[1] * xg[1] + bbar[2] * xg[2];
        double val = q0 + chi * pv + om * low;
        double r0 = chi * p1 + om * bbar[0], r1 = chi * p2 + om * bbar[1], r2 = chi * p3 + om * bbar[2];
        double out[4];
        out[0] = val;
#pragma unroll
        for (int r = 0; r < 3; ++r) out[1 + r] = JiT[r][0] * r0 + JiT[r][1] * r1 + JiT[r][2] * r2;
        const int m = g >> 2, kk = g & 3, q = m >> 1;
        // the face record of the minus-side cell: this cell's plus face, the minus neighbour's
        const int side = (m & 1) ? 0 : 1;
        const long f = gp_at(b, id.i - (side && q == 0), id.j - (side && q == 1), id.k - (side && q == 2));
        double *dst = gp + ((long)(((q * 2 + side) * 4 + kk) * 20 + v * 4)) * b.gstride + f;
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[r * b.gstride] = out[r];
    }
}

// copy of the Gauss-point buffer into the per-cell export layout [c][24][5][4]
template <class TG>
__global__ void __launch_bounds__(256) k_gp_export(BlockView b, long Ntot, const TG *__restrict__ gp,
                                                   double *__restrict__ out) {
    long cl = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cl >= b.N) return;
    Idx3 id = unflatten(b, cl);
    long c = b.off + cl;
    for (int g = 0; g < kNGP; ++g) {
        const int m = g >> 2, kk = g & 3, q = m >> 1;
        const int side = (m & 1) ? 0 : 1;
        const long f = gp_at(b, id.i - (side && q == 0), id.j - (side && q == 1), id.k - (side && q == 2));
        for (int v = 0; v < 5; ++v)
            for (int r = 0; r < 4; ++r)
                out[((c * kNGP + g) * 5 + v) * 4 + r] =
                    (double)gp[((long)(((q * 2 + side) * 4 + kk) * 20 + v * 4 + r)) * b.gstride + f];
    }
}

// ------------------------------------------------------------------------------------------
// accumulation + S2O4 stage update: one thread per cell
// stash [80][Ntot]: Qpre (5) = Q^n + dt L^n + dt^2/6 L_t^n, Gb (15), Lb (60)
// ------------------------------------------------------------------------------------------
template <int STAGE, class TF, bool WALLS>
__device__ inline void update_cell(const BlockView &b, long cl, long Ntot, const TF *__restrict__ fo, const Metrics &M,
                                   const double dt, double *__restrict__ Q, double *__restrict__ G,
                                   double *__restrict__ L, double *__restrict__ stash, const TF *__restrict__ wf,
                                   long Wtot) {
    Idx3 id = unflatten(b, cl);
    const long c = b.off + cl;
    double Lf[5] = {0, 0, 0, 0, 0}, Lt[5] = {0, 0, 0, 0, 0};
    double Gq[5][3], Gt[5][3];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int r = 0; r < 3; ++r) Gq[v][r] = Gt[v][r] = 0.0;
    const double iv = 1.0 / M.vol[c];
    double qb[5];  // cell averages (stage 1: removed from the surface integral of the gradient)
#pragma unroll
    for (int v = 0; v < 5; ++v) qb[v] = (STAGE == 1) ? Q[v * Ntot + c] : 0.0;
#pragma unroll 1
    for (int q = 0; q < 3; ++q) {
        int o[3] = {0, 0, 0};
        o[q] = -1;
        const long fm = cell_at(b, id.i + o[0], id.j + o[1], id.k + o[2]);
#pragma unroll 1
        for (int kk = 0; kk < 4; ++kk) {
            const TF *Dp = fo + (long)((q * 4 + kk) * 30) * Ntot + c;   // plus face: this cell is left
            const TF *Dm = fo + (long)((q * 4 + kk) * 30) * Ntot + fm;  // minus face: this cell is right
            // F and F_t of the minus face: from the wall-face buffer at a minus-side wall
            const TF *DmF = Dm;
            long sF = Ntot;
            if constexpr (WALLS) {
                const int iq = (q == 0) ? id.i : (q == 1) ? id.j : id.k;
                if (((b.wall >> (2 * q)) & 1) && iq == 0) {
                    DmF = wf + (long)(kk * 10) * Wtot + b.wbase[q] + wall_face_index(b, q, id.i, id.j, id.k);
                    sF = Wtot;
                }
            }
            const double wp = M.fw[(q * 4 + kk) * Ntot + c], wm = M.fw[(q * 4 + kk) * Ntot + fm];
            double np_[3], nm_[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                np_[r] = M.fn[((q * 4 + kk) * 3 + r) * Ntot + c];
                nm_[r] = M.fn[((q * 4 + kk) * 3 + r) * Ntot + fm];
            }
            const int s = 4 * q + kk;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                if (STAGE == 1) {
                    Lf[v] += wm * (double)DmF[v * sF] - wp * (double)Dp[v * Ntot];
                }
                Lt[v] += wm * (double)DmF[(5 + v) * sF] - wp * (double)Dp[(5 + v) * Ntot];
                const double dqp = (double)Dp[(15 + v) * Ntot], dqm = (double)Dm[(25 + v) * Ntot];
#pragma unroll
                for (int r = 0; r < 3; ++r) Gt[v][r] += wp * np_[r] * dqp - wm * nm_[r] * dqm;
                const double lt = dqp - dqm;
                if (STAGE == 1) {
                    const double qp = (double)Dp[(10 + v) * Ntot], qm = (double)Dm[(20 + v) * Ntot];
                    // Gauss's theorem on the closed cell surface with the cell average removed
#pragma unroll
                    for (int r = 0; r < 3; ++r)
                        Gq[v][r] += wp * np_[r] * (qp - qb[v]) - wm * nm_[r] * (qm - qb[v]);
                    const double lb = qp - qm;
                    __builtin_nontemporal_store(lb, stash + ((20 + 12 * v + s) * Ntot + c));
                    L[(12 * v + s) * Ntot + c] = lb + 0.5 * dt * lt;
                } else {
                    L[(12 * v + s) * Ntot + c] = stash[(20 + 12 * v + s) * Ntot + c] + dt * lt;
                }
            }
        }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        if (STAGE == 1) {
            const double l1 = Lf[v] * iv, l2 = Lt[v] * iv, qn = qb[v];
            __builtin_nontemporal_store(qn + dt * l1 + (dt * dt / 6.0) * l2, stash + (v * Ntot + c));
            Q[v * Ntot + c] = qn + 0.5 * dt * l1 + 0.125 * dt * dt * l2;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const double gb = Gq[v][r] * iv;
                __builtin_nontemporal_store(gb, stash + ((5 + 3 * v + r) * Ntot + c));
                G[(3 * v + r) * Ntot + c] = gb + 0.5 * dt * (Gt[v][r] * iv);
            }
        } else {
            Q[v * Ntot + c] = stash[v * Ntot + c] + (dt * dt / 3.0) * (Lt[v] * iv);
#pragma unroll
            for (int r = 0; r < 3; ++r)
                G[(3 * v + r) * Ntot + c] = stash[(5 + 3 * v + r) * Ntot + c] + dt * (Gt[v][r] * iv);
        }
    }
}

// A unit is one tile; thread t updates cell t of the tile.
template <int STAGE, class TF, bool WALLS>
__global__ void __launch_bounds__(256) k_update(WorkList W, long Ntot, const TF *__restrict__ fo, Metrics M,
                                                const double *__restrict__ dtp, double *__restrict__ Q,
                                                double *__restrict__ G, double *__restrict__ L,
                                                double *__restrict__ stash, const TF *__restrict__ wf, long Wtot) {
    const double dt = *dtp;
    for (UnitRange ur = unit_range(W.ntiles, W.xcd); ur.u < ur.end; ur.u += ur.step) {
        const Tile tile = W.tiles[ur.u];
        if ((int)threadIdx.x >= tile.count) continue;
        update_cell<STAGE, TF, WALLS>(W.blocks[tile.blk], tile.start + threadIdx.x, Ntot, fo, M, dt, Q, G, L, stash,
                                      wf, Wtot);
    }
}

// explicit instantiations through launch wrappers --------------------------------------------
hipError_t launch_metrics(const BlockView &b, const double *nodes, const Metrics &M, long Ntot, int *bad, hipStream_t s) {
    dim3 grid((unsigned)((b.N + 255) / 256));
    hipLaunchKernelGGL(k_metrics, grid, dim3(256), 0, s, b, nodes, M, Ntot, bad);
    return hipGetLastError();
}

hipError_t launch_dt(long off, long N, long Ntot, const double *Q, const double *dtm, const DevParams &P,
                     double *part, int nparts, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_dt_partial, dim3(nparts), dim3(256), 0, s, off, N, Ntot, Q, dtm, P, part, flag);
    return hipGetLastError();
}

hipError_t launch_diagnostics(long Ntot, const double *Q, const double *G, const double *vol, const DevParams &P,
                              double *part, int nparts, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_partial, dim3(nparts), dim3(256), 0, s, Ntot, Q, G, vol, P, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, part, nparts, out);
    return hipGetLastError();
}

hipError_t launch_dt_final(const double *part, int n, double *dt, hipStream_t s) {
    hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(256), 0, s, part, n, dt);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// flow diagnostics from the compact reconstruction (3^3 Gauss points per cell)
// ------------------------------------------------------------------------------------------
// Coefficients of every cell and variable of a periodic block into coef [v][kDiagCoef][Ntot]:
// a (34), chi, bbar (3).
constexpr int kDiagCoef = kNB + 4;
__global__ void __launch_bounds__(256) k_diag_coeffs(BlockView b, long Ntot, const double *__restrict__ Q,
                                                     const double *__restrict__ G, const double *__restrict__ L,
                                                     Metrics M, const DevConsts *__restrict__ K, DevParams P,
                                                     double *__restrict__ coef) {
    const long cl = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cl >= b.N) return;
    const int v = blockIdx.y;
    const long c = b.off + cl;
    double q0, a[kNB], chi, bbar[3];
    valu_coeffs(b, Ntot, Q, G, L, M, K, P, cl, v, q0, a, chi, bbar);
    double *dst = coef + (long)v * kDiagCoef * Ntot + c;
#pragma unroll
    for (int r = 0; r < kNB; ++r) dst[r * Ntot] = a[r];
    dst[kNB * Ntot] = chi;
#pragma unroll
    for (int t = 0; t < 3; ++t) dst[(kNB + 1 + t) * Ntot] = bbar[t];
}

// Partial sums of a periodic block's cells over the 27 Gauss points of each cell (the sums of
// k_diag_partial), at the points' reconstructed states: values chi P^4 + (1 - chi)(Q_0 +
// bbar . xi), reference gradients likewise, physical gradients by (J0^T)^-1, volume element
// |det J| of the cell's trilinear map at the point.  One workgroup per part, the cells of the
// block in a fixed order.
__global__ void __launch_bounds__(256) k_diag_hq_partial(BlockView b, long Ntot, const double *__restrict__ Q,
                                                         const double *__restrict__ coef,
                                                         const double *__restrict__ nodes, Metrics M,
                                                         const DevConsts *__restrict__ K, DevParams P,
                                                         double *__restrict__ part) {
    __shared__ double red[kDiagVals][256];
    double acc[kDiagVals] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, INFINITY};
    for (long cl = (long)blockIdx.x * blockDim.x + threadIdx.x; cl < b.N; cl += (long)gridDim.x * blockDim.x) {
        const Idx3 id = unflatten(b, cl);
        const long c = b.off + cl;
        const double *Pn[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) Pn[t] = node_ptr(nodes, b, id.i + (t & 1), id.j + ((t >> 1) & 1), id.k + (t >> 2));
        double JiT[3][3], q0[5], chi[5], bb[5][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q) JiT[r][q] = M.JiT[(3 * r + q) * Ntot + c];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double *cv = coef + (long)v * kDiagCoef * Ntot + c;
            q0[v] = Q[v * Ntot + c];
            chi[v] = cv[kNB * Ntot];
#pragma unroll
            for (int t = 0; t < 3; ++t) bb[v][t] = cv[(kNB + 1 + t) * Ntot];
        }
#pragma unroll 1
        for (int g = 0; g < kVolGP; ++g) {
            const double *xi = K->xv[g];
            // trilinear map on the centred cell [-1/2, 1/2]^3: Jacobian at xi
            double Jm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int ci = t & 1, cj = (t >> 1) & 1, ck = t >> 2;
                const double f0 = ci ? 0.5 + xi[0] : 0.5 - xi[0], f1 = cj ? 0.5 + xi[1] : 0.5 - xi[1],
                             f2 = ck ? 0.5 + xi[2] : 0.5 - xi[2];
                const double d0 = ci ? 1.0 : -1.0, d1 = cj ? 1.0 : -1.0, d2 = ck ? 1.0 : -1.0;
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    Jm[r][0] += Pn[t][r] * d0 * f1 * f2;
                    Jm[r][1] += Pn[t][r] * f0 * d1 * f2;
                    Jm[r][2] += Pn[t][r] * f0 * f1 * d2;
                }
            }
            const double det = Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) -
                               Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0]) +
                               Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]);
            const double dV = K->wv[g] * fabs(det);
            double qv[5], gr[5][3];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double *cv = coef + (long)v * kDiagCoef * Ntot + c;
                double pv = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll 2
                for (int r = 0; r < kNB; ++r) {
                    const double a = cv[r * Ntot];
                    pv = fma(K->V[g][0][r], a, pv);
                    p1 = fma(K->V[g][1][r], a, p1);
                    p2 = fma(K->V[g][2][r], a, p2);
                    p3 = fma(K->V[g][3][r], a, p3);
                }
                const double om = 1.0 - chi[v];
                qv[v] = q0[v] + chi[v] * pv + om * (bb[v][0] * xi[0] + bb[v][1] * xi[1] + bb[v][2] * xi[2]);
                const double r0 = chi[v] * p1 + om * bb[v][0], r1 = chi[v] * p2 + om * bb[v][1],
                             r2 = chi[v] * p3 + om * bb[v][2];
#pragma unroll
                for (int r = 0; r < 3; ++r) gr[v][r] = JiT[r][0] * r0 + JiT[r][1] * r1 + JiT[r][2] * r2;
            }
            const double rho = qv[0];
            double U[3], uu = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                U[d] = qv[1 + d] / rho;
                uu += U[d] * U[d];
            }
            const double kin = 0.5 * rho * uu;
            const double p = (P.gamma - 1.0) * (qv[4] - kin);
            const double mu = viscosity_dt(P, p / rho);
            double dU[3][3];
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int e = 0; e < 3; ++e) dU[d][e] = (gr[1 + d][e] - U[d] * gr[0][e]) / rho;
            const double w0 = dU[2][1] - dU[1][2], w1 = dU[0][2] - dU[2][0], w2 = dU[1][0] - dU[0][1];
            acc[0] += dV;
            acc[1] += rho * dV;
            acc[2] += kin * dV;
            acc[3] += mu * (w0 * w0 + w1 * w1 + w2 * w2) * dV;
            acc[4] += qv[4] * dV;
            acc[5] = fmin(acc[5], rho);
            acc[6] = fmin(acc[6], p);
        }
    }
#pragma unroll
    for (int i = 0; i < kDiagVals; ++i) red[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int i = 0; i < 5; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + h];
#pragma unroll
            for (int i = 5; i < kDiagVals; ++i) red[i][threadIdx.x] = fmin(red[i][threadIdx.x], red[i][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < kDiagVals) part[(long)blockIdx.x * kDiagVals + threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_diagnostics_hq(const BlockView &b, long Ntot, const double *Q, const double *G, const double *L,
                                 const double *nodes, const Metrics &M, const DevConsts *K, const DevParams &P,
                                 double *coef, double *part, int nparts, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_coeffs, dim3((unsigned)((b.N + 255) / 256), 5), dim3(256), 0, s, b, Ntot, Q, G, L, M, K,
                       P, coef);
    hipLaunchKernelGGL(k_diag_hq_partial, dim3((unsigned)nparts), dim3(256), 0, s, b, Ntot, Q, coef, nodes, M, K, P,
                       part);
    return hipGetLastError();
}

hipError_t launch_diagnostics_final(const double *part, int nparts, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, part, nparts, out);
    return hipGetLastError();
}

hipError_t launch_recon(const BlockView &b, long Ntot, const double *Q, const double *G, const double *L,
                        const Metrics &M, const DevConsts *K, const DevParams &P, double *gp, hipStream_t s) {
    dim3 grid((unsigned)((b.N + 255) / 256), 5);
    hipLaunchKernelGGL(k_recon, grid, dim3(256), 0, s, b, Ntot, Q, G, L, M, K, P, gp);
    return hipGetLastError();
}

hipError_t launch_gp_export(bool gp32, const BlockView &b, long Ntot, const void *gp, double *out, hipStream_t s) {
    dim3 grid((unsigned)((b.N + 255) / 256));
    if (gp32)
        hipLaunchKernelGGL(k_gp_export<float>, grid, dim3(256), 0, s, b, Ntot, (const float *)gp, out);
    else
        hipLaunchKernelGGL(k_gp_export<double>, grid, dim3(256), 0, s, b, Ntot, (const double *)gp, out);
    return hipGetLastError();
}

static dim3 work_grid(long units, int ngroups) {
    return dim3((unsigned)((ngroups <= 0 || ngroups > units) ? units : ngroups));
}

hipError_t launch_update(int stage, bool fo32, const WorkList &W, long Ntot, const void *fo, const Metrics &M,
                         const double *dt, double *Q, double *G, double *L, double *stash, int ngroups,
                         const void *wf, long Wtot, hipStream_t s) {
    // wf: the wall-face buffer, or NULL for work lists of periodic blocks only.  The stage-1
    // update runs in its wall-capable form for every block: with the per-face redirect
    // (not taken without walls) it measured faster than the periodic form, 14.4 against 16.2
    // ms at 256^3 (the periodic form unrolled over the four Gauss points of a face; without
    // the unroll it was slower still), with bitwise equal results.
    if (W.ntiles <= 0) return hipSuccess;
    const dim3 grid = work_grid(W.ntiles, ngroups), bl(kUpdateTile);
#define CGKS_UPDATE(ST, TF, WL)                                                                                   \
    hipLaunchKernelGGL((k_update<ST, TF, WL>), grid, bl, 0, s, W, Ntot, (const TF *)fo, M, dt, Q, G, L, stash, \
                       (const TF *)wf, Wtot)
    if (fo32) {
        // stage 1 in the wall-capable form here too (its code measured faster, as for FP64)
        if (stage == 1) CGKS_UPDATE(1, float, true);
        else if (wf) CGKS_UPDATE(2, float, true);
        else CGKS_UPDATE(2, float, false);
    } else {
        if (stage == 1) CGKS_UPDATE(1, double, true);
        else if (wf) CGKS_UPDATE(2, double, true);
        else CGKS_UPDATE(2, double, false);
    }
#undef CGKS_UPDATE
    return hipGetLastError();
}

}  // namespace cgks
