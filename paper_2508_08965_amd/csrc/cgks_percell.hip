// Reconstruction with per-cell stored matrices: the comparison baseline for the shared
// standard-cell matrix (Sec. 4, last paragraph).
//
// Without the standard cell, every cell needs its own linear maps, because the frame in which
// its stencil data enter differs from cell to cell.  This variant stores them per cell:
//   Rc  (34 x 84)  polynomial coefficients from the cell's raw stencil data in the physical
//                  frame: face and edge average differences (6 + 12), the physical gradients
//                  of the face and edge neighbours (18 + 36) and the line derivatives (12);
//                  Rc = R T_c with T_c the cell's frame transform of the stencil data (J0^T for
//                  the gradients, tau . J0^T for the edge directional derivatives)
//   Ec  (96 x 34)  value and physical gradient at the 24 face Gauss points: the value rows of
//                  E and the gradient rows of E back-transformed with the cell's (J0^T)^-1
// that is 6120 doubles (48,960 bytes) per cell.  Storage is tiled by the 64 cells a wave takes:
// tile t = cell / 64 holds element e of its cells at ((t * 6120 + e) * 64 + cell % 64), with Rc
// column-major (e = 34 j + i) and Ec after it (e = 2856 + 34 (4 g + r) + i), so that one load of
// a wave reads 512 consecutive bytes at a constant offset from the lane's tile base.  The
// smoothness indicators keep the shared Gram
// matrices (they act on the standard-cell coefficients) and the blend is the one of the other
// reconstruction kernels, so all three produce the same Gauss-point values up to rounding.
//
// One lane per (cell, conserved variable): a workgroup is one wave, 64 cells of one variable.
// The five workgroups of a tile (one per variable) get numbers 8 apart, which places them on the
// same XCD, so that the four after the first find the tile's matrices in that XCD's L2.
#include <hip/hip_runtime.h>

#include "cgks_device.h"

namespace cgks {

namespace {

__device__ inline long pc_cell(const BlockView &b, int i, int j, int k) {
    i = (i < 0) ? i + b.nx : (i >= b.nx ? i - b.nx : i);
    j = (j < 0) ? j + b.ny : (j >= b.ny ? j - b.ny : j);
    k = (k < 0) ? k + b.nz : (k >= b.nz ? k - b.nz : k);
    return b.off + (long)i + (long)b.nx * ((long)j + (long)b.ny * k);
}

// edge n of the cell: axes pa < pb with offsets sa, sb; pc the third axis (same numbering as
// the stencil rows of the standard-cell system)
__device__ inline void edge_axes(int n, int &pa, int &pb, int &pc, int &sa, int &sb) {
    pa = (n < 8) ? 0 : 1;
    pb = (n < 4) ? 1 : 2;
    pc = 3 - pa - pb;
    sa = (n & 1) ? 1 : -1;
    sb = (n & 2) ? 1 : -1;
}

}  // namespace

// Per-cell matrices of one block: one thread per cell.
__global__ void __launch_bounds__(256) k_percell_setup(BlockView b, long Ntot, Metrics M,
                                                       const DevConsts *__restrict__ K, double *__restrict__ pcm) {
    const long cl = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cl >= b.N) return;
    const long c = b.off + cl;
    double J0[3][3], JiT[3][3];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
            J0[r][q] = M.J0[(3 * r + q) * Ntot + c];
            JiT[r][q] = M.JiT[(3 * r + q) * Ntot + c];
        }
    double *t = pcm + (c / kPcTile) * kPcElems * kPcTile + c % kPcTile;
    auto rc = [&](int i, int j) -> double & { return t[(long)(j * kNB + i) * kPcTile]; };
    const double is2 = 0.70710678118654752440;
#pragma unroll 1
    for (int i = 0; i < kNB; ++i) {
        const double *Ri = K->R[i];
        for (int m = 0; m < 6; ++m) rc(i, m) = Ri[m];
        for (int n = 0; n < 12; ++n) rc(i, 6 + n) = Ri[kRowEdgeAvg + n];
        for (int m = 0; m < 6; ++m)
            for (int k = 0; k < 3; ++k) {
                double s = 0.0;
                for (int j = 0; j < 3; ++j) s += Ri[kRowFaceGrad + 3 * m + j] * J0[k][j];
                rc(i, 18 + 3 * m + k) = s;
            }
        for (int n = 0; n < 12; ++n) {
            int pa, pb, pc, sa, sb;
            edge_axes(n, pa, pb, pc, sa, sb);
            for (int k = 0; k < 3; ++k)
                rc(i, 36 + 3 * n + k) =
                    Ri[kRowEdgeDir + 2 * n] * J0[k][pc] + Ri[kRowEdgeDir + 2 * n + 1] * (sa * J0[k][pa] + sb * J0[k][pb]) * is2;
        }
        for (int s = 0; s < 12; ++s) rc(i, 72 + s) = Ri[kRowLine + s];
    }
    double *ec = t + (long)kNB * kPcCols * kPcTile;
#pragma unroll 1
    for (int g = 0; g < kNGP; ++g)
        for (int i = 0; i < kNB; ++i) {
            ec[(long)((g * 4) * kNB + i) * kPcTile] = K->E[g][0][i];
            for (int r = 0; r < 3; ++r)
                ec[(long)((g * 4 + 1 + r) * kNB + i) * kPcTile] =
                    JiT[r][0] * K->E[g][1][i] + JiT[r][1] * K->E[g][2][i] + JiT[r][2] * K->E[g][3][i];
        }
}

__global__ void __launch_bounds__(64) k_recon_percell(BlockView b, long Ntot, const double *__restrict__ Q,
                                                       const double *__restrict__ G, const double *__restrict__ L,
                                                       Metrics M, const DevConsts *__restrict__ K, DevParams P,
                                                       const double *__restrict__ pcm, double *__restrict__ gp) {
    // the Gram matrices of the smoothness indicators, staged once per workgroup
    __shared__ double sGL[kNB * kNB], sGT[kNB * kNB];
    for (int i = threadIdx.x; i < kNB * kNB; i += blockDim.x) {
        sGL[i] = (&K->GL[0][0])[i];
        sGT[i] = (&K->GT[0][0])[i];
    }
    __syncthreads();
    // workgroup w -> (tile, variable): w = ((tile / 8) * 5 + v) * 8 + tile % 8
    const int w = blockIdx.x, v = (w >> 3) % 5;
    const long tile_b = (long)((w >> 3) / 5) * 8 + (w & 7);
    const long cl = tile_b * kPcTile + threadIdx.x;
    if (cl >= b.N) return;
    const int ci = (int)(cl % b.nx), cj = (int)((cl / b.nx) % b.ny), ck = (int)(cl / ((long)b.nx * b.ny));
    const long c = b.off + cl;
    const double *Qv = Q + v * Ntot;
    const double *Gv = G + 3 * v * Ntot;
    const double *Lv = L + 12 * v * Ntot;
    const double q0 = Qv[c];

    // a = Rc r, one stencil item r_j at a time (column j of the cell's matrix)
    double a[kNB];
#pragma unroll
    for (int i = 0; i < kNB; ++i) a[i] = 0.0;
    const double *tile = pcm + (c / kPcTile) * kPcElems * kPcTile + c % kPcTile;
    auto column = [&](int j, double x) {
        const double *col = tile + j * kNB * kPcTile;
#pragma unroll
        for (int i = 0; i < kNB; ++i) a[i] = fma(col[i * kPcTile], x, a[i]);
    };
    double fd[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        int o[3] = {0, 0, 0};
        o[m >> 1] = (m & 1) ? 1 : -1;
        const long nb = pc_cell(b, ci + o[0], cj + o[1], ck + o[2]);
        fd[m] = Qv[nb] - q0;
        column(m, fd[m]);
#pragma unroll
        for (int k = 0; k < 3; ++k) column(18 + 3 * m + k, Gv[k * Ntot + nb]);
    }
#pragma unroll
    for (int n = 0; n < 12; ++n) {
        int pa, pb, pc, sa, sb;
        edge_axes(n, pa, pb, pc, sa, sb);
        int o[3] = {0, 0, 0};
        o[pa] = sa;
        o[pb] = sb;
        const long nb = pc_cell(b, ci + o[0], cj + o[1], ck + o[2]);
        column(6 + n, Qv[nb] - q0);
#pragma unroll
        for (int k = 0; k < 3; ++k) column(36 + 3 * n + k, Gv[k * Ntot + nb]);
    }
    double lines[12];
#pragma unroll
    for (int s = 0; s < 12; ++s) {
        lines[s] = Lv[s * Ntot + c];
        column(72 + s, lines[s]);
    }

    // low-order blend: linear polynomials of the six face sub-stencils and their weights
    double bbar[3] = {0.0, 0.0, 0.0}, chi = 1.0;
    if (!P.linear) {
        double lm[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) lm[t] = 0.25 * (lines[4 * t] + lines[4 * t + 1] + lines[4 * t + 2] + lines[4 * t + 3]);
        double wsum = 0.0, wv[6], bm[6][3];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const int q = m >> 1;
#pragma unroll
            for (int t = 0; t < 3; ++t) bm[m][t] = (t == q) ? ((m & 1) ? fd[m] : -fd[m]) : lm[t];
            const double is = bm[m][0] * bm[m][0] + bm[m][1] * bm[m][1] + bm[m][2] * bm[m][2] + P.geno_eps;
            const double is2 = is * is;
            wv[m] = (1.0 / 6.0) / (is2 * is2 * is);
            wsum += wv[m];
        }
        const double iw = 1.0 / wsum;
#pragma unroll
        for (int m = 0; m < 6; ++m)
#pragma unroll
            for (int t = 0; t < 3; ++t) bbar[t] += (wv[m] * iw) * bm[m][t];
        // smoothness indicators on the standard-cell coefficients (shared Gram matrices)
        double isl = 0.0, ist = 0.0;
#pragma unroll
        for (int r = 0; r < kNB; ++r) {
            double tl = 0.0, tt = 0.0;
#pragma unroll
            for (int s = 0; s < kNB; ++s) {
                tl = fma(sGL[r * kNB + s], a[s], tl);
                tt = fma(sGT[r * kNB + s], a[s], tt);
            }
            isl = fma(a[r], tl, isl);
            ist = fma(a[r], tt, ist);
            __builtin_amdgcn_sched_barrier(0);
        }
        const double ish = isl + ist;
        const double rh = ist / (ish + P.geno_eps), rl = ist / (isl + P.geno_eps);
        double ah, al;
        if (P.geno_r == 2.0) {
            ah = 1.0 + rh * rh;
            al = 1.0 + rl * rl;
        } else {
            ah = 1.0 + pow(rh, P.geno_r);
            al = 1.0 + pow(rl, P.geno_r);
        }
        chi = tanh(P.geno_C * (2.0 * ah / (ah + al))) * P.inv_tanhC;
    }
    // the low-order gradient bbar is in the standard-cell frame: back-transform it once
    double jb[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        jb[r] = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) jb[r] += M.JiT[(3 * r + q) * Ntot + c] * bbar[q];
    }
    const double om = 1.0 - chi;
#pragma unroll 1
    for (int g = 0; g < kNGP; ++g) {
        const double *eg = tile + (long)(kNB * kPcCols + g * 4 * kNB) * kPcTile;
        double p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int i = 0; i < kNB; ++i) p[r] = fma(eg[(r * kNB + i) * kPcTile], a[i], p[r]);
        }
        const double *xg = K->xg[g];
        const double low = bbar[0] * xg[0] + bbar[1] * xg[1] + bbar[2] * xg[2];
        const int m = g >> 2, kk = g & 3, q = m >> 1;
        // the face record of the minus-side cell: this cell's plus face, the minus neighbour's
        const int side = (m & 1) ? 0 : 1;
        const long f = gp_at(b, ci - (side && q == 0), cj - (side && q == 1), ck - (side && q == 2));
        double *dst = gp + ((long)(((q * 2 + side) * 4 + kk) * 20 + v * 4)) * b.gstride + f;
        dst[0] = q0 + chi * p[0] + om * low;
#pragma unroll
        for (int r = 0; r < 3; ++r) dst[(1 + r) * b.gstride] = chi * p[1 + r] + om * jb[r];
    }
}

hipError_t launch_percell_setup(const BlockView &b, long Ntot, const Metrics &M, const DevConsts *K, double *pcm,
                                hipStream_t s) {
    const dim3 grid((unsigned)((b.N + 255) / 256));
    hipLaunchKernelGGL(k_percell_setup, grid, dim3(256), 0, s, b, Ntot, M, K, pcm);
    return hipGetLastError();
}

hipError_t launch_recon_percell(const BlockView &b, long Ntot, const double *Q, const double *G, const double *L,
                                const Metrics &M, const DevConsts *K, const DevParams &P, const double *pcm,
                                double *gp, hipStream_t s) {
    const long tiles = (b.N + kPcTile - 1) / kPcTile;
    const dim3 grid((unsigned)(((tiles + 7) / 8) * 8 * 5));  // tiles padded to a multiple of 8, x 5 variables
    hipLaunchKernelGGL(k_recon_percell, grid, dim3(kPcTile), 0, s, b, Ntot, Q, G, L, M, K, P, pcm, gp);
    return hipGetLastError();
}

}  // namespace cgks
