// Device-side structures and the gas-kinetic flux of one Gauss point (FP64).
#pragma once

#include <hip/hip_runtime.h>

#include "cgks_internal.h"

namespace cgks {

struct BlockView {
    int nx, ny, nz;
    long N;    // cells of the block
    long off;  // offset of the block's first cell in the concatenated state
};

// Per-cell metrics, SoA with stride Ntot.
struct Metrics {
    double *vol;  // [Ntot]
    double *J0;   // [9][Ntot]  row-major dx_i/dxi_j
    double *JiT;  // [9][Ntot]  (J0^T)^-1 row-major
    double *fn;   // [3 axis][4 GP][3][Ntot] unit normal of the plus face
    double *fw;   // [3][4][Ntot] Gauss weight times area element
    double *dtm;  // [3 axis][4][Ntot] mean unit normal (3) and 1/h of the axis
};

struct DevConsts {
    double R[kNB][kNR];
    double E[kNGP][4][kNB];
    double GL[kNB][kNB];
    double GT[kNB][kNB];
    double xg[kNGP][3];
};

// ------------------------------------------------------------------------------------------
// Maxwellian moments.  For a Maxwellian with macroscopic velocity (U,V,W) and lambda,
// normalised to unit density: u-moments over the full line or a half line, v- and w-moments,
// and the internal-energy moments <xi^0>, <xi^2>, <xi^4> of K internal degrees of freedom.
// ------------------------------------------------------------------------------------------
struct Moments {
    double u[7], v[6], w[6], x[3];
};

__device__ inline void line_moments(double c, double i2l, double *m, int n) {
    // <x^0> = 1, <x^1> = c, <x^{k+2}> = c <x^{k+1}> + (k+1)/(2 lambda) <x^k>
    m[0] = 1.0;
    m[1] = c;
    for (int k = 0; k + 2 < n; ++k) m[k + 2] = c * m[k + 1] + (k + 1) * i2l * m[k];
}

// half: +1 -> u > 0, -1 -> u < 0, 0 -> full line
__device__ inline void maxwell_moments(double U, double V, double W, double lam, double K, int half, Moments &M) {
    const double i2l = 0.5 / lam;
    if (half == 0) {
        line_moments(U, i2l, M.u, 7);
    } else {
        const double sl = sqrt(lam);
        const double h0 = 0.5 * erfc(-half * sl * U);
        const double ex = 0.5 * exp(-lam * U * U) / (sl * 1.7724538509055160273);  // / sqrt(pi lam)
        M.u[0] = h0;
        M.u[1] = U * h0 + half * ex;
        for (int k = 0; k + 2 < 7; ++k) M.u[k + 2] = U * M.u[k + 1] + (k + 1) * i2l * M.u[k];
    }
    line_moments(V, i2l, M.v, 6);
    line_moments(W, i2l, M.w, 6);
    M.x[0] = 1.0;
    M.x[1] = K * i2l;
    M.x[2] = K * (K + 2.0) * i2l * i2l;
}

// Packed symmetric 5x5 matrix  S_{ij} = < psi_i psi_j u^A v^B w^C >,
// psi = (1, u, v, w, (u^2 + v^2 + w^2 + xi^2)/2).  Index of (i <= j): kSym[i][j].
__device__ constexpr int kSym[5][5] = {{0, 1, 2, 3, 4}, {1, 5, 6, 7, 8}, {2, 6, 9, 10, 11}, {3, 7, 10, 12, 13}, {4, 8, 11, 13, 14}};

template <int A, int B, int C>
__device__ inline void psi_matrix(const Moments &m, double S[15]) {
    auto e = [&](int p, int q, int r, int s) { return m.u[A + p] * m.v[B + q] * m.w[C + r] * m.x[s]; };
    S[0] = e(0, 0, 0, 0);
    S[1] = e(1, 0, 0, 0);
    S[2] = e(0, 1, 0, 0);
    S[3] = e(0, 0, 1, 0);
    S[5] = e(2, 0, 0, 0);
    S[6] = e(1, 1, 0, 0);
    S[7] = e(1, 0, 1, 0);
    S[9] = e(0, 2, 0, 0);
    S[10] = e(0, 1, 1, 0);
    S[12] = e(0, 0, 2, 0);
    // psi_i * psi_4
    S[4] = 0.5 * (e(2, 0, 0, 0) + e(0, 2, 0, 0) + e(0, 0, 2, 0) + e(0, 0, 0, 1));
    S[8] = 0.5 * (e(3, 0, 0, 0) + e(1, 2, 0, 0) + e(1, 0, 2, 0) + e(1, 0, 0, 1));
    S[11] = 0.5 * (e(2, 1, 0, 0) + e(0, 3, 0, 0) + e(0, 1, 2, 0) + e(0, 1, 0, 1));
    S[13] = 0.5 * (e(2, 0, 1, 0) + e(0, 2, 1, 0) + e(0, 0, 3, 0) + e(0, 0, 1, 1));
    S[14] = 0.25 * (e(4, 0, 0, 0) + e(0, 4, 0, 0) + e(0, 0, 4, 0) + e(0, 0, 0, 2)) +
            0.5 * (e(2, 2, 0, 0) + e(2, 0, 2, 0) + e(2, 0, 0, 1) + e(0, 2, 2, 0) + e(0, 2, 0, 1) + e(0, 0, 2, 1));
}

// y (+)= scale * S x
__device__ inline void sym_mv_acc(const double S[15], const double x[5], double scale, double y[5]) {
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 5; ++j) s = fma(S[kSym[i][j]], x[j], s);
        y[i] = fma(scale, s, y[i]);
    }
}

// Solve <psi psi^T> x = b for the Maxwellian (U,V,W,lambda) in closed form.
__device__ inline void slope_solve(const double b[5], double U, double V, double W, double lam, double K, double x[5]) {
    const double B = U * U + V * V + W * W + (K + 3.0) * 0.5 / lam;
    const double r2 = b[1] - U * b[0], r3 = b[2] - V * b[0], r4 = b[3] - W * b[0];
    const double r5 = 2.0 * b[4] - B * b[0];
    x[4] = 4.0 * lam * lam / (K + 3.0) * (r5 - 2.0 * (U * r2 + V * r3 + W * r4));
    x[1] = 2.0 * lam * r2 - U * x[4];
    x[2] = 2.0 * lam * r3 - V * x[4];
    x[3] = 2.0 * lam * r4 - W * x[4];
    x[0] = b[0] - U * x[1] - V * x[2] - W * x[3] - 0.5 * B * x[4];
}

__device__ inline double dev_viscosity(const DevParams &P, double T) {
    if (!P.visc_law) return P.mu0;
    double r = T / P.T_ref;
    return P.mu0 * r * sqrt(r) * (P.T_ref + P.S_suth) / (T + P.S_suth);
}

// Time integrals over [0,T] of the six coefficients of the interface distribution.
__device__ inline void time_integrals(double T, double tau, double C[6]) {
    if (tau == 0.0) {
        C[0] = T;
        C[1] = 0.0;
        C[2] = 0.5 * T * T;
        C[3] = C[4] = C[5] = 0.0;
        return;
    }
    const double e = exp(-T / tau), ome = 1.0 - e;
    C[0] = T - tau * ome;
    C[1] = 2.0 * tau * tau * ome - tau * T * (1.0 + e);
    C[2] = 0.5 * T * T - tau * T + tau * tau * ome;
    C[3] = tau * ome;
    C[4] = 2.0 * tau * tau * ome - tau * T * e;
    C[5] = tau * tau * ome;
}

__device__ inline double pair_swap(double v) { return __shfl_xor(v, 1, 64); }

// Gas-kinetic flux of one Gauss point evaluated by a lane pair (see cgks_flux in cgks.h for
// the contract).  Lane parity sd = 0 holds the left state, sd = 1 the right state; both lanes
// of the pair must be active.  Each lane builds the slopes, the time-derivative coefficient
// and the half-space moment sums of its own side; the sums are exchanged, and the equilibrium
// part is split without divergence: the even lane evaluates the moments <psi ...> (interface
// state), the odd lane the moments <u psi ...> (flux), by running the same code on u-moments
// shifted by sd.  Outputs of lane sd: its one-sided interface value and time derivative
// (Qs, dQs); the odd lane also returns F^n and F_t^n (Fo, Fto) in the global frame.
// Returns a non-zero mask (1 rho <= 0, 2 p <= 0, 4 non-finite) for non-physical input.
__device__ inline int gks_flux_pair(const DevParams &P, const int sd, const double q[5], const double g[5][3],
                                    const double n[3], const double dt, double Fo[5], double Fto[5], double Qs[5],
                                    double dQs[5]) {
    const double gam = P.gamma, K = P.K;
    double t1[3];
    if (fabs(n[0]) > fabs(n[2])) {
        const double r = 1.0 / sqrt(n[0] * n[0] + n[1] * n[1]);
        t1[0] = -n[1] * r; t1[1] = n[0] * r; t1[2] = 0.0;
    } else {
        const double r = 1.0 / sqrt(n[1] * n[1] + n[2] * n[2]);
        t1[0] = 0.0; t1[1] = -n[2] * r; t1[2] = n[1] * r;
    }
    const double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
    const double *fr[3] = {n, t1, t2};
    int err = 0;

    // ---- own side: state and directional derivatives in the face frame -----------------
    double Wk[5], a[3][5];
    Wk[0] = q[0];
    Wk[4] = q[4];
#pragma unroll
    for (int d = 0; d < 3; ++d) Wk[1 + d] = fr[d][0] * q[1] + fr[d][1] * q[2] + fr[d][2] * q[3];
    const double r = Wk[0], ir = 1.0 / r;
    const double U = Wk[1] * ir, V = Wk[2] * ir, W = Wk[3] * ir;
    const double p = (gam - 1.0) * (Wk[4] - 0.5 * r * (U * U + V * V + W * W));
    if (!(r > 0.0)) err |= 1;
    if (!(p > 0.0)) err |= 2;
    const double lm = 0.5 * r / p;
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        double dv[5], bb[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) dv[v] = fr[dir][0] * g[v][0] + fr[dir][1] * g[v][1] + fr[dir][2] * g[v][2];
        bb[0] = dv[0] * ir;
        bb[4] = dv[4] * ir;
#pragma unroll
        for (int d = 0; d < 3; ++d) bb[1 + d] = (fr[d][0] * dv[1] + fr[d][1] * dv[2] + fr[d][2] * dv[3]) * ir;
        slope_solve(bb, U, V, W, lm, K, a[dir]);
    }
    double Ak[5], dWk[5];
    {
        Moments mf;
        maxwell_moments(U, V, W, lm, K, 0, mf);
        double S[15], rhs[5] = {0, 0, 0, 0, 0};
        psi_matrix<1, 0, 0>(mf, S); sym_mv_acc(S, a[0], -1.0, rhs);
        psi_matrix<0, 1, 0>(mf, S); sym_mv_acc(S, a[1], -1.0, rhs);
        psi_matrix<0, 0, 1>(mf, S); sym_mv_acc(S, a[2], -1.0, rhs);
        slope_solve(rhs, U, V, W, lm, K, Ak);
#pragma unroll
        for (int v = 0; v < 5; ++v) dWk[v] = r * rhs[v];
    }
    // half-space moment sums of this side: X[0] W0, X[1..3] dW0 per direction, then
    // fh0 <u psi>, fh1 <u psi a.u>, fh2 <u psi A>, wh1 <psi a.u>, wh2 <psi A> (times rho)
    double X[9][5];
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int v = 0; v < 5; ++v) X[i][v] = 0.0;
    {
        Moments mh;
        maxwell_moments(U, V, W, lm, K, sd ? -1 : 1, mh);
        double S[15];
        psi_matrix<0, 0, 0>(mh, S);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            X[0][v] = r * S[kSym[v][0]];
            X[4][v] = r * S[kSym[v][1]];
        }
#pragma unroll
        for (int dir = 0; dir < 3; ++dir) sym_mv_acc(S, a[dir], r, X[1 + dir]);
        sym_mv_acc(S, Ak, r, X[8]);
        psi_matrix<1, 0, 0>(mh, S);
        sym_mv_acc(S, Ak, r, X[6]);
        sym_mv_acc(S, a[0], r, X[7]);
        psi_matrix<0, 1, 0>(mh, S); sym_mv_acc(S, a[1], r, X[7]);
        psi_matrix<0, 0, 1>(mh, S); sym_mv_acc(S, a[2], r, X[7]);
        psi_matrix<2, 0, 0>(mh, S); sym_mv_acc(S, a[0], r, X[5]);
        psi_matrix<1, 1, 0>(mh, S); sym_mv_acc(S, a[1], r, X[5]);
        psi_matrix<1, 0, 1>(mh, S); sym_mv_acc(S, a[2], r, X[5]);
    }
    // pair sums (a + b is exact-order independent, so both lanes hold identical totals)
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int v = 0; v < 5; ++v) X[i][v] += pair_swap(X[i][v]);
    const double p_other = pair_swap(p);
    err |= __shfl_xor(err, 1, 64);

    // ---- equilibrium state at the interface --------------------------------------------
    const double r0 = X[0][0], ir0 = 1.0 / r0;
    const double U0 = X[0][1] * ir0, V0 = X[0][2] * ir0, Z0 = X[0][3] * ir0;
    const double p0 = (gam - 1.0) * (X[0][4] - 0.5 * r0 * (U0 * U0 + V0 * V0 + Z0 * Z0));
    if (!(r0 > 0.0)) err |= 1;
    if (!(p0 > 0.0)) err |= 2;
    const double lam0 = 0.5 * r0 / p0;
    double ab[3][5];
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        double bb[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) bb[v] = X[1 + dir][v] * ir0;
        slope_solve(bb, U0, V0, Z0, lam0, K, ab[dir]);
    }
    // u-moments shifted by sd: psi-moments on the even lane, u psi-moments on the odd lane
    Moments m0;
    {
        double us[8];
        line_moments(U0, 0.5 / lam0, us, 8);
#pragma unroll
        for (int k = 0; k < 7; ++k) m0.u[k] = sd ? us[k + 1] : us[k];
        line_moments(V0, 0.5 / lam0, m0.v, 6);
        line_moments(Z0, 0.5 / lam0, m0.w, 6);
        m0.x[0] = 1.0;
        m0.x[1] = K * 0.5 / lam0;
        m0.x[2] = K * (K + 2.0) * 0.25 / (lam0 * lam0);
    }
    double e1[5] = {0, 0, 0, 0, 0}, e0v[5], e2[5] = {0, 0, 0, 0, 0}, Ab[5];
    {
        double S[15];
        psi_matrix<1, 0, 0>(m0, S); sym_mv_acc(S, ab[0], 1.0, e1);
        psi_matrix<0, 1, 0>(m0, S); sym_mv_acc(S, ab[1], 1.0, e1);
        psi_matrix<0, 0, 1>(m0, S); sym_mv_acc(S, ab[2], 1.0, e1);
        // time-derivative coefficient of g0 from the compatibility condition: needs the
        // psi-moment (even lane) version of e1
        double rhs[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double o = pair_swap(e1[v]);
            rhs[v] = -(sd ? o : e1[v]);
        }
        slope_solve(rhs, U0, V0, Z0, lam0, K, Ab);
        psi_matrix<0, 0, 0>(m0, S);
#pragma unroll
        for (int v = 0; v < 5; ++v) e0v[v] = S[kSym[v][0]];
        sym_mv_acc(S, Ab, 1.0, e2);
    }
    // collision time (Sec. 5)
    double tau;
    if (P.tau_zero) {
        tau = 0.0;
    } else {
        const double jump = fabs((p - p_other) / (p + p_other));
        tau = P.viscous ? dev_viscosity(P, p0 * ir0) / p0 + P.tau_C * jump * dt : (P.tau_eps + P.tau_C * jump) * dt;
    }
    double C1[6], C2[6];
    time_integrals(dt, tau, C1);
    time_integrals(0.5 * dt, tau, C2);
    const double idt = 1.0 / dt;
    double cn[6], ct[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        cn[i] = (4.0 * C2[i] - C1[i]) * idt;
        ct[i] = 4.0 * (C1[i] - 2.0 * C2[i]) * idt * idt;
    }
    // even lane: interface state W^n, W_t^n;  odd lane: flux F^n, F_t^n (face frame)
    double Yn[5], Yt[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const double h0 = sd ? X[4][v] : X[0][v];
        const double h1 = sd ? X[5][v] : X[7][v];
        const double h2 = sd ? X[6][v] : X[8][v];
        Yn[v] = r0 * (cn[0] * e0v[v] + cn[1] * e1[v] + cn[2] * e2[v]) + cn[3] * h0 - cn[4] * h1 - cn[5] * h2;
        Yt[v] = r0 * (ct[0] * e0v[v] + ct[1] * e1[v] + ct[2] * e2[v]) + ct[3] * h0 - ct[4] * h1 - ct[5] * h2;
    }
    double Wn[5], Wt[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const double on = pair_swap(Yn[v]), ot = pair_swap(Yt[v]);
        Wn[v] = sd ? on : Yn[v];
        Wt[v] = sd ? ot : Yt[v];
    }
    if (P.viscous && P.prandtl_fix && !P.tau_zero) {
        // heat flux relative to the interface velocity, corrected to Pr (odd lane holds F)
        const double uu = U0 * U0 + V0 * V0 + Z0 * Z0, kf = 1.0 / P.Pr - 1.0;
        const double qn = Yn[4] - (U0 * Yn[1] + V0 * Yn[2] + Z0 * Yn[3]) + 0.5 * uu * Yn[0] - U0 * Wn[4] +
                          U0 * (U0 * Wn[1] + V0 * Wn[2] + Z0 * Wn[3]) - 0.5 * U0 * uu * Wn[0];
        const double qt = Yt[4] - (U0 * Yt[1] + V0 * Yt[2] + Z0 * Yt[3]) + 0.5 * uu * Yt[0] - U0 * Wt[4] +
                          U0 * (U0 * Wt[1] + V0 * Wt[2] + Z0 * Wt[3]) - 0.5 * U0 * uu * Wt[0];
        if (sd) {
            Yn[4] += kf * qn;
            Yt[4] += kf * qt;
        }
    }
    // one-sided interface values (tau0 = tau)
    const double e0 = (tau > 0.0) ? exp(-dt / tau) : 0.0, oe = 1.0 - e0;
    double Sq[5], St[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        Sq[v] = oe * Wn[v] + e0 * Wk[v];
        St[v] = oe * Wt[v] + e0 * dWk[v];
    }
    // back to the global frame
    Qs[0] = Sq[0]; Qs[4] = Sq[4];
    dQs[0] = St[0]; dQs[4] = St[4];
    Fo[0] = Yn[0]; Fo[4] = Yn[4];
    Fto[0] = Yt[0]; Fto[4] = Yt[4];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Qs[1 + c] = n[c] * Sq[1] + t1[c] * Sq[2] + t2[c] * Sq[3];
        dQs[1 + c] = n[c] * St[1] + t1[c] * St[2] + t2[c] * St[3];
        Fo[1 + c] = n[c] * Yn[1] + t1[c] * Yn[2] + t2[c] * Yn[3];
        Fto[1 + c] = n[c] * Yt[1] + t1[c] * Yt[2] + t2[c] * Yt[3];
    }
    bool finite = true;
#pragma unroll
    for (int v = 0; v < 5; ++v) finite = finite && isfinite(Fo[v]) && isfinite(Fto[v]) && isfinite(Qs[v]) && isfinite(dQs[v]);
    if (!finite) err |= 4;
    return err;
}

// launch wrappers (cgks_kernels.hip)
hipError_t launch_metrics(const BlockView &b, const double *nodes, const Metrics &M, long Ntot, int *bad, hipStream_t s);
hipError_t launch_dt(long off, long N, long Ntot, const double *Q, const double *dtm, const DevParams &P,
                     double *part, int nparts, int *flag, hipStream_t s);
hipError_t launch_dt_final(const double *part, int n, double *dt, hipStream_t s);
hipError_t launch_recon(const BlockView &b, long Ntot, const double *Q, const double *G, const double *L,
                        const Metrics &M, const DevConsts *K, const DevParams &P, double *gp, hipStream_t s);
hipError_t launch_recon_mfma(const BlockView &b, long Ntot, const double *Q, const double *G, const double *L,
                             const Metrics &M, const double *Kblk, const DevParams &P, double *gp, int ngroups,
                             hipStream_t s);
hipError_t launch_gp_export(const BlockView &b, long Ntot, const double *gp, double *out, hipStream_t s);
hipError_t launch_flux(const BlockView &b, long Ntot, const double *gp, const Metrics &M, const double *dt,
                       const DevParams &P, double *fo, int *flag, hipStream_t s);
hipError_t launch_flux_points(long n, const double *ql, const double *gl, const double *qr, const double *gr,
                              const double *nrm, const double *dt, const DevParams &P, double *F, double *Ft,
                              double *S, int *flag, hipStream_t s);
hipError_t launch_update(int stage, const BlockView &b, long Ntot, const double *fo, const Metrics &M,
                         const double *dt, double *Q, double *G, double *L, double *stash, hipStream_t s);

}  // namespace cgks
