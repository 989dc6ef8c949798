// HIP kernels of the gas-kinetic flux at the face Gauss points (Sec. 2, eq. flux, linearisation)
// for gfx950, with their launch wrappers:
//
//   k_flux        : every owned face of the work list, two lanes per Gauss point
//   k_flux_wall   : the faces on wall sides of one block (symmetry, no-slip, far field,
//                   non-reflecting), after k_flux
//   k_flux_points : the flux of independent Gauss-point states (cgks_flux)
//
// This file is compiled on its own, with the scheduler's AMDGPU register-pressure trackers
// (-mllvm -amdgpu-use-amdgpu-trackers): with them the FP64 flux, at 2 waves per SIMD, fits its
// 256 VGPRs without the 28 / 12 bytes of spill the default scheduling leaves (stage 1 about 4 %
// faster at 256^3), while the same option slows the stage-1 update with FP32 face records, which
// stays in cgks_kernels.hip.
//
// Data layout as in cgks_kernels.hip:
//   gp  [q][side][k][v*4 + c][Gtot]   reconstructed value (c = 0) and physical gradient
//                                     (c = 1..3) at Gauss point k of face q of the face record
//                                     owned by the minus-side cell (cells at gp_at(), rows
//                                     padded to 16 cells)
//   fo  [q][k][30][Ntot]              F^n (5), F_t^n (5), Q^l, dQ^l/dt, Q^r, dQ^r/dt (20)
#include <hip/hip_runtime.h>

#include "cgks_device.h"

namespace cgks {

// ------------------------------------------------------------------------------------------
// gas-kinetic flux kernels
// ------------------------------------------------------------------------------------------
// Two lanes per Gauss point.  A unit is (tile, owned-face Gauss point qk = 4q + kk); thread t of
// the workgroup serves cell t / 2 of the tile (the face record of its plus face), side t & 1.
// POS: each side's state is first limited toward its own cell's average (positivity_state);
// the cell of the right side is the +q neighbour of the record's cell, periodic in its block.
template <class TC, class TG, class TF, bool FULL, bool POS = false>
__global__ void __launch_bounds__(256, 2) k_flux(WorkList W, long Ntot, const TG *__restrict__ gp, Metrics M,
                                              const double *__restrict__ dtp, DevParams P,
                                              TF *__restrict__ fo, int *__restrict__ flag, const double *__restrict__ Q) {
    const long u = unit_once((long)W.ntiles * 12, W.xcd);
    if (u < 0) return;
    const Tile tile = W.tiles[u / 12];
    const int qk = (int)(u % 12), q = qk >> 2, kk = qk & 3;
    const int i = (int)(threadIdx.x >> 1), sd = (int)(threadIdx.x & 1);
    if (i >= tile.count) return;  // both lanes of a pair leave together
    const BlockView &bk = W.blocks[tile.blk];
    const long f = bk.off + tile.start + i;
    TC qv[5], gv[5][3], n[3];
    const long gs = bk.gstride;
    const TG *src = gp + (long)(((q * 2 + sd) * 4 + kk) * 20) * gs + gp_local(bk, tile.start + i);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        qv[v] = (TC)src[(4 * v) * gs];
#pragma unroll
        for (int j = 0; j < 3; ++j) gv[v][j] = (TC)src[(4 * v + 1 + j) * gs];
    }
    if constexpr (POS) {
        long own = f;
        if (sd) {
            const BlockView &b = W.blocks[tile.blk];
            const long l = tile.start + i, nxy = (long)b.nx * b.ny;
            int ci = (int)(l % b.nx), cj = (int)((l / b.nx) % b.ny), ck = (int)(l / nxy);
            if (q == 0) ci = (ci + 1 == b.nx) ? 0 : ci + 1;
            else if (q == 1) cj = (cj + 1 == b.ny) ? 0 : cj + 1;
            else ck = (ck + 1 == b.nz) ? 0 : ck + 1;
            own = b.off + ci + (long)b.nx * cj + nxy * ck;
        }
        double qb[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) qb[v] = Q[v * Ntot + own];
        positivity_state<TC>(P, qb, qv, gv);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) n[r] = (TC)M.fn[((q * 4 + kk) * 3 + r) * Ntot + f];
    TC F[5], Ft[5], Qs[5], dQs[5];
    const int bad = gks_flux_pair<DevMath, TC, FULL>(P, sd, qv, gv, n, (TC)*dtp, F, Ft, Qs, dQs);
    if (bad && sd == 0) atomicOr(flag, bad);
    TF *dst = fo + (long)((q * 4 + kk) * 30) * Ntot + f;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        // the second stage's update reads only the time derivatives F_t and dQ/dt
        if constexpr (FULL) dst[(10 + 10 * sd + v) * Ntot] = (TF)Qs[v];
        dst[(15 + 10 * sd + v) * Ntot] = (TF)dQs[v];
        if (sd) {
            if constexpr (FULL) dst[v * Ntot] = (TF)F[v];
            dst[(5 + v) * Ntot] = (TF)Ft[v];
        }
    }
}

// Wall faces of axis q of one block, two lanes per Gauss point.  A pair serves (wall face p,
// Gauss point kk, wall w: 0 minus side, 1 plus side).  The face record f of the cell at index
// n_q - 1 (the plus wall) holds the Gauss-point data of both walls of its line: its left side is
// that cell's, its right side was written by the cell at index 0 (the minus wall).  Both lanes
// load the interior side; the ghost lane (left at the minus wall, right at the plus wall)
// mirrors its copy across the wall.  The plus wall's flux replaces the record's F, F_t and left
// side values; the minus wall's replaces the record's right side values and puts F, F_t into
// the wall-face buffer wf [(kk 10 + item)][Wtot].  At a no-slip wall the mass and energy
// components of F and F_t are zero (impermeable, at rest, adiabatic).  Runs after k_flux.
template <class TC, class TG, class TF, bool FULL>
__global__ void __launch_bounds__(256) k_flux_wall(BlockView b, int q, long Ntot, const TG *__restrict__ gp, Metrics M,
                                                   const double *__restrict__ dtp, DevParams P, TF *__restrict__ fo,
                                                   TF *__restrict__ wf, long Wtot, int *__restrict__ flag) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long pair = t >> 1;
    const int sd = (int)(t & 1);
    const long nfaces = b.N / ((q == 0) ? b.nx : (q == 1) ? b.ny : b.nz);
    const long p = pair >> 3;
    if (p >= nfaces) return;  // both lanes of a pair leave together
    const int kk = (int)((pair >> 1) & 3), w = (int)(pair & 1);
    int i, j, k;
    if (q == 0) {
        i = b.nx - 1; j = (int)(p % b.ny); k = (int)(p / b.ny);
    } else if (q == 1) {
        i = (int)(p % b.nx); j = b.ny - 1; k = (int)(p / b.nx);
    } else {
        i = (int)(p % b.nx); j = (int)(p / b.nx); k = b.nz - 1;
    }
    const long f = b.off + i + (long)b.nx * (j + (long)b.ny * k);
    const int side = 2 * q + w;
    TC qv[5], gv[5][3], n[3];
    const TG *src = gp + (long)(((q * 2 + (1 - w)) * 4 + kk) * 20) * b.gstride + gp_at(b, i, j, k);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        qv[v] = (TC)src[(4 * v) * b.gstride];
#pragma unroll
        for (int r = 0; r < 3; ++r) gv[v][r] = (TC)src[(4 * v + 1 + r) * b.gstride];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) n[r] = (TC)M.fn[((q * 4 + kk) * 3 + r) * Ntot + f];
    if (sd == w) {
        if ((b.wall >> (24 + side)) & 1) {
            // non-reflecting: the characteristic boundary state of the interior one (outward
            // normal: n at the plus wall, -n at the minus wall), with the interior gradient
            const TC no[3] = {w ? n[0] : -n[0], w ? n[1] : -n[1], w ? n[2] : -n[2]};
            TC qb[5];
            nonreflecting_state<TC>((TC)P.gamma, P.far, qv, no, qb);
#pragma unroll
            for (int v = 0; v < 5; ++v) qv[v] = qb[v];
        } else {
            const bool far = (b.wall >> (16 + side)) & 1;  // far field: the uniform far-field state
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const TC m = (TC)mirror_sign(b.wall, side, v);
                qv[v] = far ? (TC)P.far[v] : qv[v] * m;
#pragma unroll
                for (int r = 0; r < 3; ++r) gv[v][r] = far ? (TC)0 : ((r == q) ? -m : m) * gv[v][r];
            }
        }
    }
    TC F[5], Ft[5], Qs[5], dQs[5];
    const int bad = gks_flux_pair<DevMath, TC, FULL>(P, sd, qv, gv, n, (TC)*dtp, F, Ft, Qs, dQs);
    if (bad && sd == 0) atomicOr(flag, bad);
    if ((b.wall >> (8 + side)) & 1) F[0] = F[4] = Ft[0] = Ft[4] = (TC)0;
    TF *dst = fo + (long)((q * 4 + kk) * 30) * Ntot + f;
    if (sd != w) {  // the interior lane: its one-sided values
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            if constexpr (FULL) dst[(10 + 10 * sd + v) * Ntot] = (TF)Qs[v];
            dst[(15 + 10 * sd + v) * Ntot] = (TF)dQs[v];
        }
    }
    if (sd) {
        TF *fd = w ? dst : wf + (long)(kk * 10) * Wtot + b.wbase[q] + p;
        const long st = w ? Ntot : Wtot;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            if constexpr (FULL) fd[v * st] = (TF)F[v];
            fd[(5 + v) * st] = (TF)Ft[v];
        }
    }
}

template <class TC>
__global__ void __launch_bounds__(256) k_flux_points(long n, const double *__restrict__ ql_, const double *__restrict__ gl_,
                                                     const double *__restrict__ qr_, const double *__restrict__ gr_,
                                                     const double *__restrict__ nrm, const double *__restrict__ dtp,
                                                     DevParams P, double *__restrict__ F_, double *__restrict__ Ft_,
                                                     double *__restrict__ S_, int *__restrict__ flag) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long i = t >> 1;
    if (i >= n) return;
    const int sd = (int)(t & 1);
    const double *q_ = sd ? qr_ : ql_;
    const double *g_ = sd ? gr_ : gl_;
    TC qv[5], gv[5][3], nn[3];
    for (int v = 0; v < 5; ++v) {
        qv[v] = (TC)q_[5 * i + v];
        for (int j = 0; j < 3; ++j) gv[v][j] = (TC)g_[15 * i + 3 * v + j];
    }
    for (int r = 0; r < 3; ++r) nn[r] = (TC)nrm[3 * i + r];
    TC F[5], Ft[5], Qs[5], dQs[5];
    const int bad = gks_flux_pair<DevMath, TC>(P, sd, qv, gv, nn, (TC)*dtp, F, Ft, Qs, dQs);
    if (bad && sd == 0) atomicOr(flag, bad);
    for (int v = 0; v < 5; ++v) {
        S_[20 * i + 10 * sd + v] = Qs[v];
        S_[20 * i + 10 * sd + 5 + v] = dQs[v];
        if (sd) {
            F_[5 * i + v] = F[v];
            Ft_[5 * i + v] = Ft[v];
        }
    }
}

// launch wrappers ---------------------------------------------------------------------------
hipError_t launch_flux(int flux_prec, bool gp32, const WorkList &W, long Ntot, const void *gp, const Metrics &M,
                       const double *dt, const DevParams &P, void *fo, int *flag, bool full, const double *Q,
                       hipStream_t s) {
    if (W.ntiles <= 0) return hipSuccess;
    const long units = (long)W.ntiles * 12;
    const dim3 grid((unsigned)(W.xcd ? 8 * ((units + 7) / 8) : units));
    const bool pos = P.positivity != 0;
#define CGKS_FLUX_ONE(TC, TG, TF, FULL, POS)                                                               \
    hipLaunchKernelGGL((k_flux<TC, TG, TF, FULL, POS>), grid, dim3(2 * kFluxTile), 0, s, W, Ntot,        \
                       (const TG *)gp, M, dt, P, (TF *)fo, flag, Q)
#define CGKS_FLUX(TC, TG, TF)                                                                              \
    do {                                                                                                   \
        if (full && !pos) CGKS_FLUX_ONE(TC, TG, TF, true, false);                                          \
        else if (full) CGKS_FLUX_ONE(TC, TG, TF, true, true);                                              \
        else if (!pos) CGKS_FLUX_ONE(TC, TG, TF, false, false);                                            \
        else CGKS_FLUX_ONE(TC, TG, TF, false, true);                                                       \
    } while (0)
    if (flux_prec == 0 && !gp32)
        CGKS_FLUX(double, double, double);
    else if (flux_prec == 0)
        CGKS_FLUX(double, float, double);
    else
        CGKS_FLUX(float, float, float);
#undef CGKS_FLUX
#undef CGKS_FLUX_ONE
    return hipGetLastError();
}

hipError_t launch_flux_points(int flux_prec, long n, const double *ql, const double *gl, const double *qr,
                              const double *gr, const double *nrm, const double *dt, const DevParams &P, double *F,
                              double *Ft, double *S, int *flag, hipStream_t s) {
    dim3 grid((unsigned)((2 * n + 255) / 256));
    if (flux_prec == 0)
        hipLaunchKernelGGL(k_flux_points<double>, grid, dim3(256), 0, s, n, ql, gl, qr, gr, nrm, dt, P, F, Ft, S, flag);
    else
        hipLaunchKernelGGL(k_flux_points<float>, grid, dim3(256), 0, s, n, ql, gl, qr, gr, nrm, dt, P, F, Ft, S, flag);
    return hipGetLastError();
}

hipError_t launch_flux_wall(int flux_prec, bool gp32, const BlockView &b, int q, long Ntot, const void *gp,
                            const Metrics &M, const double *dt, const DevParams &P, void *fo, void *wf, long Wtot,
                            int *flag, bool full, hipStream_t s) {
    const long nfaces = b.N / ((q == 0) ? b.nx : (q == 1) ? b.ny : b.nz);
    const long threads = nfaces * 16;  // 4 Gauss points x 2 walls x 2 lanes per face
    const dim3 grid((unsigned)((threads + 255) / 256)), bl(256);
#define CGKS_FLUXW(TC, TG, TF)                                                                                   \
    do {                                                                                                         \
        if (full)                                                                                                \
            hipLaunchKernelGGL((k_flux_wall<TC, TG, TF, true>), grid, bl, 0, s, b, q, Ntot, (const TG *)gp, M,   \
                               dt, P, (TF *)fo, (TF *)wf, Wtot, flag);                                           \
        else                                                                                                     \
            hipLaunchKernelGGL((k_flux_wall<TC, TG, TF, false>), grid, bl, 0, s, b, q, Ntot, (const TG *)gp, M,  \
                               dt, P, (TF *)fo, (TF *)wf, Wtot, flag);                                           \
    } while (0)
    if (flux_prec == 0 && !gp32)
        CGKS_FLUXW(double, double, double);
    else if (flux_prec == 0)
        CGKS_FLUXW(double, float, double);
    else
        CGKS_FLUXW(float, float, float);
#undef CGKS_FLUXW
    return hipGetLastError();
}

}  // namespace cgks
