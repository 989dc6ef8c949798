// Device-side structures and the gas-kinetic flux of one Gauss point (FP64).
#pragma once

#include <hip/hip_runtime.h>

#include "cgks_internal.h"

namespace cgks {

// Meshes hold fewer than kMaxCells cells in total, so that a cell index and the byte offset of
// an element of one component array (index x 8) fit in 32 bits.
constexpr long kMaxCells = 1L << 27;

struct BlockView {
    int nx, ny, nz;
    long N;    // cells of the block
    long off;  // offset of the block's first cell in the concatenated state
    // Sides s = 2q + (0 minus, 1 plus) of axis q: bit s marks a non-periodic side (symmetry
    // plane, no-slip wall, far field or non-reflecting), bit 8 + s a no-slip wall, bit 16 + s a
    // far-field side, bit 24 + s a non-reflecting side; 0 for a periodic block.  Non-periodic
    // sides come in pairs per axis.
    int wall;
    // Per axis with walls: offset of the block's minus-side wall faces in the wall-face buffer
    // (one entry per face of that side, index i_a + n_a i_b over the tangential axes a < b).
    long wbase[3];
    // Gauss-point buffer: cell (i, j, k) of the block at goff + i + nxp (j + ny k), rows padded
    // to nxp = nx rounded up to 16 cells and goff a multiple of 16, so that every row of 16
    // cells the reconstruction writes starts on a 128-byte boundary; gstride: the buffer's
    // stride between components (the same for every block).
    long goff, gstride;
    int nxp;
};

// Index in the Gauss-point buffer of cell (i, j, k) of block b, periodic in the block.
__host__ __device__ inline long gp_at(const BlockView &b, int i, int j, int k) {
    i = (i < 0) ? i + b.nx : (i >= b.nx ? i - b.nx : i);
    j = (j < 0) ? j + b.ny : (j >= b.ny ? j - b.ny : j);
    k = (k < 0) ? k + b.nz : (k >= b.nz ? k - b.nz : k);
    return b.goff + (long)i + (long)b.nxp * ((long)j + (long)b.ny * k);
}
// Index in the Gauss-point buffer of the block-local linear cell index l.
__host__ __device__ inline long gp_local(const BlockView &b, long l) {
    return (b.nxp == b.nx) ? b.goff + l : b.goff + l % b.nx + (long)b.nxp * (l / b.nx);
}

// Sign of conserved variable v in the mirror image across wall side s: the momentum normal to
// a symmetry plane, and every momentum component at a no-slip wall, change sign.
__host__ __device__ inline double mirror_sign(int wall, int s, int v) {
    if ((wall >> (24 + s)) & 1) return 1.0;  // non-reflecting side: no mirror image
    return (v >= 1 && v <= 3 && (((wall >> (8 + s)) & 1) || v - 1 == (s >> 1))) ? -1.0 : 1.0;
}

// Boundary state of a non-reflecting side: locally one-dimensional characteristics along the
// outward unit normal n.  The Riemann invariant u_n + 2c/(gamma - 1) leaves the domain with
// the interior state q, u_n - 2c/(gamma - 1) enters with the far-field state f; with the
// normal velocity and sound speed these fix, entropy p/rho^gamma and tangential velocity come
// from q at an outflow and from f at an inflow.  Supersonic outflow: q; supersonic inflow: f.
template <class T>
__device__ inline void nonreflecting_state(T gam, const double *f, const T q[5], const T n[3], T qb[5]) {
    const T gm1 = gam - T(1);
    T ui[3], ue[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        ui[r] = q[1 + r] / q[0];
        ue[r] = (T)f[1 + r] / (T)f[0];
    }
    const T pi = gm1 * (q[4] - T(0.5) * q[0] * (ui[0] * ui[0] + ui[1] * ui[1] + ui[2] * ui[2]));
    const T pe = gm1 * ((T)f[4] - T(0.5) * (T)f[0] * (ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2]));
    const T ci = sqrt(gam * pi / q[0]), ce = sqrt(gam * pe / (T)f[0]);
    const T uni = ui[0] * n[0] + ui[1] * n[1] + ui[2] * n[2];
    const T une = ue[0] * n[0] + ue[1] * n[1] + ue[2] * n[2];
    if (uni >= ci) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qb[v] = q[v];
        return;
    }
    if (uni <= -ci) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qb[v] = (T)f[v];
        return;
    }
    const T rout = uni + T(2) * ci / gm1, rin = une - T(2) * ce / gm1;
    const T unb = T(0.5) * (rout + rin), cb = T(0.25) * gm1 * (rout - rin);
    const bool out = unb > T(0);
    const T rho_s = out ? q[0] : (T)f[0], p_s = out ? pi : pe, un_s = out ? uni : une;
    const T cs2 = gam * p_s / rho_s;
    const T rhob = rho_s * pow(cb * cb / cs2, T(1) / gm1);
    const T pb = rhob * cb * cb / gam;
    T k = T(0);
    qb[0] = rhob;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const T ub = (out ? ui[r] : ue[r]) + (unb - un_s) * n[r];
        qb[1 + r] = rhob * ub;
        k += ub * ub;
    }
    qb[4] = pb / gm1 + T(0.5) * rhob * k;
}

// Index of a wall face of axis q within its side: i_a + n_a i_b over the tangential axes.
__host__ __device__ inline long wall_face_index(const BlockView &b, int q, int i, int j, int k) {
    return (q == 0) ? (long)j + (long)b.ny * k : (q == 1) ? (long)i + (long)b.nx * k : (long)i + (long)b.nx * j;
}

// A run of consecutive cells of one block (block-local linear index, x fastest): the unit of
// the work lists that let one launch cover every block of a multi-block mesh.
// A tile is either a run of consecutive cells (ty = 0; every kernel) or, for the
// reconstruction, a brick of count x ty x tz cells whose corner cell is `start` (rows of the
// brick are split into chunks of 16 cells along x, planes are visited in order of z so that a
// workgroup re-reads the neighbour planes it has just touched).
struct Tile {
    int blk;     // index into the block table
    int count;   // cells in the run (>= 1), or x extent of the brick
    long start;  // first cell of the run, or corner cell of the brick (block-local)
    int ty, tz;  // brick extents in y and z (0 for a run)
    int pad0, pad1;
};

struct WorkList {
    const BlockView *blocks;  // device table, one entry per block
    const Tile *tiles;        // device, ntiles entries
    int ntiles;
    int xcd;  // 1: the workgroups of XCD x (w mod 8 == x) share the x-th contiguous eighth of the units
};

// Units [u, end) with stride `step` of the calling workgroup.  Workgroups are dispatched to the
// 8 XCDs round-robin, so with xcd set (and a grid that is a multiple of 8) each XCD walks a
// contiguous eighth of the list and keeps the neighbours of its cells in its own L2.
struct UnitRange {
    long u, end, step;
};

#ifdef __HIPCC__
__device__ inline UnitRange unit_range(long nunits, int xcd) {
    const long G = gridDim.x, w = blockIdx.x;
    if (xcd && G >= 8 && (G & 7) == 0) {
        const long x = w & 7, G8 = G >> 3;
        return {nunits * x / 8 + (w >> 3), nunits * (x + 1) / 8, G8};
    }
    return {w, nunits, G};
}

// The one unit of a workgroup in a grid of 8 ceil(nunits / 8) (xcd set) or nunits workgroups;
// -1 for the padding workgroups of the XCD order.
__device__ inline long unit_once(long nunits, int xcd) {
    const long w = blockIdx.x;
    if (!xcd) return w;
    const long x = w & 7, u = nunits * x / 8 + (w >> 3);
    return u < nunits * (x + 1) / 8 ? u : -1;
}
#endif

// Per-cell metrics, SoA with stride Ntot.
struct Metrics {
    double *vol;  // [Ntot]
    double *J0;   // [9][Ntot]  row-major dx_i/dxi_j
    double *JiT;  // [9][Ntot]  (J0^T)^-1 row-major
    double *fn;   // [3 axis][4 GP][3][Ntot] unit normal of the plus face
    double *fw;   // [3][4][Ntot] Gauss weight times area element
    double *dtm;  // [3 axis][4][Ntot] mean unit normal (3) and 1/h of the axis
};

constexpr int kVolGP = 27;  // 3^3 Gauss points of the volume integrals of the diagnostics
struct DevConsts {
    double R[kNB][kNR];
    double E[kNGP][4][kNB];
    double GL[kNB][kNB];
    double GT[kNB][kNB];
    double xg[kNGP][3];
    double V[kVolGP][4][kNB];  // basis value and reference gradient at the volume Gauss points
    double xv[kVolGP][3];      // the volume Gauss points (centred standard cell), x fastest
    double wv[kVolGP];         // their weights (sum 1)
};

// ------------------------------------------------------------------------------------------
// Gas-kinetic flux, generic in the arithmetic type T (double on the FP64 path, float on the
// FP32 flux path, an operation-counting type in the host op-count tool).  Pair exchange and
// math functions are supplied by the policy class X:
//   X::swap(v)  value of v held by the partner lane of the pair (lane id xor 1)
//   X::sqrt, X::exp, X::erfc, X::fabs, X::fma, X::finite, X::pow
// ------------------------------------------------------------------------------------------
// Partner-lane exchange as a DPP register move (quad_perm [1,0,3,2], i.e. lane id xor 1)
// rather than through LDS.  Both lanes of every pair are active wherever it is used.
__device__ inline int pair_swap32(int v) { return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false); }

struct DevMath {
    __device__ static double swap(double v) {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = (unsigned)pair_swap32((int)(unsigned)b);
        const unsigned hi = (unsigned)pair_swap32((int)(unsigned)(b >> 32));
        return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
    }
    __device__ static float swap(float v) { return __builtin_bit_cast(float, pair_swap32(__builtin_bit_cast(int, v))); }
    __device__ static int swapi(int v) { return pair_swap32(v); }
    template <class T> __device__ static T sqrt(T x) { return ::sqrt(x); }
    template <class T> __device__ static T exp(T x) { return ::exp(x); }
    template <class T> __device__ static T erfc(T x) { return ::erfc(x); }
    template <class T> __device__ static T fabs(T x) { return ::fabs(x); }
    template <class T> __device__ static T fma(T a, T b, T c) { return ::fma(a, b, c); }
    template <class T> __device__ static T pow(T a, T b) { return ::pow(a, b); }
    template <class T> __device__ static bool finite(T x) { return isfinite(x); }
    // Marks the start (true) and end (false) of work that both lanes of a pair perform
    // identically (or that only one lane's result uses); free on the device, it lets a host
    // instantiation count the flux's work once per Gauss point.
    __device__ static void pair_shared(bool) {}
};

// Maxwellian moments normalised to unit density: <u^k> over the full line or a half line,
// <v^k>, <w^k>, and <xi^0>, <xi^2>, <xi^4> of K internal degrees of freedom.
template <class T>
struct MomentsT {
    T u[7], v[6], w[6], x[3];
};

template <class T>
__host__ __device__ inline void line_moments(T c, T i2l, T *m, int n) {
    // <x^0> = 1, <x^1> = c, <x^{k+2}> = c <x^{k+1}> + (k+1)/(2 lambda) <x^k>
    m[0] = T(1.0);
    m[1] = c;
    for (int k = 0; k + 2 < n; ++k) m[k + 2] = c * m[k + 1] + T(k + 1) * i2l * m[k];
}

// half: +1 -> u > 0, -1 -> u < 0, 0 -> full line
template <class X, class T>
__host__ __device__ inline void maxwell_moments(T U, T V, T W, T lam, T i2l, T K, int half, MomentsT<T> &M) {
    if (half == 0) {
        line_moments<T>(U, i2l, M.u, 7);
    } else {
        const T sl = X::sqrt(lam);
        const T h0 = T(0.5) * X::erfc(T(-half) * sl * U);
        const T ex = T(0.5) * X::exp(-lam * U * U) / (sl * T(1.7724538509055160273));  // / sqrt(pi lam)
        M.u[0] = h0;
        M.u[1] = U * h0 + T(half) * ex;
        for (int k = 0; k + 2 < 7; ++k) M.u[k + 2] = U * M.u[k + 1] + T(k + 1) * i2l * M.u[k];
    }
    line_moments<T>(V, i2l, M.v, 6);
    line_moments<T>(W, i2l, M.w, 6);
    M.x[0] = T(1.0);
    M.x[1] = K * i2l;
    M.x[2] = K * (K + T(2.0)) * i2l * i2l;
}

// Packed symmetric 5x5 matrix  S_{ij} = < psi_i psi_j u^A v^B w^C >,
// psi = (1, u, v, w, (u^2 + v^2 + w^2 + xi^2)/2).  Index of (i <= j): sym_idx(i, j).
__host__ __device__ constexpr int sym_idx(int i, int j) {
    return (i <= j) ? (i * 5 - i * (i - 1) / 2 + (j - i)) : (j * 5 - j * (j - 1) / 2 + (i - j));
}

template <int A, int B, int C, class T>
__host__ __device__ inline void psi_matrix(const MomentsT<T> &m, T S[15]) {
    auto e = [&](int p, int q, int r, int s) { return m.u[A + p] * m.v[B + q] * m.w[C + r] * m.x[s]; };
    S[sym_idx(0, 0)] = e(0, 0, 0, 0);
    S[sym_idx(0, 1)] = e(1, 0, 0, 0);
    S[sym_idx(0, 2)] = e(0, 1, 0, 0);
    S[sym_idx(0, 3)] = e(0, 0, 1, 0);
    S[sym_idx(1, 1)] = e(2, 0, 0, 0);
    S[sym_idx(1, 2)] = e(1, 1, 0, 0);
    S[sym_idx(1, 3)] = e(1, 0, 1, 0);
    S[sym_idx(2, 2)] = e(0, 2, 0, 0);
    S[sym_idx(2, 3)] = e(0, 1, 1, 0);
    S[sym_idx(3, 3)] = e(0, 0, 2, 0);
    // psi_i * psi_4
    S[sym_idx(0, 4)] = T(0.5) * (e(2, 0, 0, 0) + e(0, 2, 0, 0) + e(0, 0, 2, 0) + e(0, 0, 0, 1));
    S[sym_idx(1, 4)] = T(0.5) * (e(3, 0, 0, 0) + e(1, 2, 0, 0) + e(1, 0, 2, 0) + e(1, 0, 0, 1));
    S[sym_idx(2, 4)] = T(0.5) * (e(2, 1, 0, 0) + e(0, 3, 0, 0) + e(0, 1, 2, 0) + e(0, 1, 0, 1));
    S[sym_idx(3, 4)] = T(0.5) * (e(2, 0, 1, 0) + e(0, 2, 1, 0) + e(0, 0, 3, 0) + e(0, 0, 1, 1));
    S[sym_idx(4, 4)] = T(0.25) * (e(4, 0, 0, 0) + e(0, 4, 0, 0) + e(0, 0, 4, 0) + e(0, 0, 0, 2)) +
                       T(0.5) * (e(2, 2, 0, 0) + e(2, 0, 2, 0) + e(2, 0, 0, 1) + e(0, 2, 2, 0) + e(0, 2, 0, 1) +
                                 e(0, 0, 2, 1));
}

// y (+)= scale * S x
template <class X, class T>
__host__ __device__ inline void sym_mv_acc(const T S[15], const T x[5], T scale, T y[5]) {
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        T s = T(0.0);
#pragma unroll
        for (int j = 0; j < 5; ++j) s = X::fma(S[sym_idx(i, j)], x[j], s);
        y[i] = X::fma(scale, s, y[i]);
    }
}

// Solve <psi psi^T> x = b for the Maxwellian (U,V,W,lambda) in closed form.  The factors that
// depend on the state only are formed once per state (each state is solved for several b).
template <class T>
struct SlopeSolver {
    T U, V, W, B, twol, c5;
    __host__ __device__ SlopeSolver(T U_, T V_, T W_, T lam, T i2l, T K, T invK3)
        : U(U_), V(V_), W(W_), B(U_ * U_ + V_ * V_ + W_ * W_ + (K + T(3.0)) * i2l), twol(T(2.0) * lam),
          c5(T(4.0) * lam * lam * invK3) {}
    __host__ __device__ void solve(const T b[5], T x[5]) const {
        const T r2 = b[1] - U * b[0], r3 = b[2] - V * b[0], r4 = b[3] - W * b[0];
        const T r5 = T(2.0) * b[4] - B * b[0];
        x[4] = c5 * (r5 - T(2.0) * (U * r2 + V * r3 + W * r4));
        x[1] = twol * r2 - U * x[4];
        x[2] = twol * r3 - V * x[4];
        x[3] = twol * r4 - W * x[4];
        x[0] = b[0] - U * x[1] - V * x[2] - W * x[3] - T(0.5) * B * x[4];
    }
};

template <class X, class T>
__host__ __device__ inline T dev_viscosity(const DevParams &P, T Tm) {
    if (!P.visc_law) return T(P.mu0);
    const T r = Tm * T(P.inv_Tref);
    return T(P.mu0) * r * X::sqrt(r) * (T(P.T_ref) + T(P.S_suth)) / (Tm + T(P.S_suth));
}

// Time integrals over [0,T] of the six coefficients of the interface distribution, given
// e = exp(-T / tau) (unused when tau_zero).
template <class X, class T>
__host__ __device__ inline void time_integrals(T Tw, T tau, T e, bool tau_zero, T C[6]) {
    if (tau_zero) {
        C[0] = Tw;
        C[1] = T(0.0);
        C[2] = T(0.5) * Tw * Tw;
        C[3] = C[4] = C[5] = T(0.0);
        return;
    }
    const T ome = T(1.0) - e;
    C[0] = Tw - tau * ome;
    C[1] = T(2.0) * tau * tau * ome - tau * Tw * (T(1.0) + e);
    C[2] = T(0.5) * Tw * Tw - tau * Tw + tau * tau * ome;
    C[3] = tau * ome;
    C[4] = T(2.0) * tau * tau * ome - tau * Tw * e;
    C[5] = tau * tau * ome;
}

// Interface-state limiter (an addition to the paper, for flows whose local Mach number reaches
// ~3 and whose internal energy is then a small part of the total): a cell's reconstructed
// state at a face Gauss point, value q and gradient g, becomes qb + theta (q - qb) and
// theta g, theta the largest value in [0, 1] keeping density and pressure at or above eps
// times those of the cell average qb.  The density bound is linear in theta; along the
// segment rho p / (gamma - 1) = rho E - |m|^2 / 2 is a quadratic a t^2 + b t + c, positive
// at t = 0, whose root in (0, 1) is 2c / (-b + sqrt(b^2 - 4ac)).  Evaluated in FP64 whatever
// the flux precision.  States at or above the floor and cells whose average is not physical
// are left as they are.
template <class T>
__host__ __device__ inline void positivity_state(const DevParams &P, const double qb[5], T q[5], T g[5][3]) {
    const double gm1 = P.gamma - 1.0;
    const double rb = qb[0];
    const double mb2 = qb[1] * qb[1] + qb[2] * qb[2] + qb[3] * qb[3];
    const double pb = gm1 * (qb[4] - 0.5 * mb2 / rb);
    if (!(rb > 0.0) || !(pb > 0.0)) return;
    const double er = P.pos_eps * rb, ep = P.pos_eps * pb;
    double th = 1.0;
    if ((double)q[0] < er) th = (rb - er) / (rb - (double)q[0]);
    double d[5], z[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        d[v] = th * ((double)q[v] - qb[v]);
        z[v] = qb[v] + d[v];
    }
    const double pz = gm1 * (z[4] - 0.5 * (z[1] * z[1] + z[2] * z[2] + z[3] * z[3]) / z[0]);
    if (pz < ep) {
        const double e1 = ep / gm1;
        const double a = d[0] * d[4] - 0.5 * (d[1] * d[1] + d[2] * d[2] + d[3] * d[3]);
        const double b = rb * d[4] + qb[4] * d[0] - (qb[1] * d[1] + qb[2] * d[2] + qb[3] * d[3]) - e1 * d[0];
        const double c = rb * qb[4] - 0.5 * mb2 - e1 * rb;
        th *= 2.0 * c / (-b + sqrt(b * b - 4.0 * a * c));
    }
    if (th < 1.0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            q[v] = (T)(qb[v] + th * ((double)q[v] - qb[v]));
#pragma unroll
            for (int r = 0; r < 3; ++r) g[v][r] = (T)(th * (double)g[v][r]);
        }
    }
}

// Gas-kinetic flux of one Gauss point evaluated by a lane pair (see cgks_flux in cgks.h for
// the contract).  Lane parity sd = 0 holds the left state, sd = 1 the right state; both lanes
// of the pair must be active.  Each lane builds the slopes, the time-derivative coefficient
// and the half-space moment sums of its own side; the sums are exchanged, and the equilibrium
// part is split without divergence: the even lane evaluates the moments <psi ...> (interface
// state), the odd lane the moments <u psi ...> (flux), by running the same code on u-moments
// shifted by sd.  Outputs of lane sd: its one-sided interface value and time derivative
// (Qs, dQs); the odd lane also returns F^n and F_t^n (Fo, Fto) in the global frame.
// Returns a non-zero mask (1 rho <= 0, 2 p <= 0, 4 non-finite) for non-physical input.
// FULL = false: only the time derivatives (Fto, dQs) are produced (the second stage's update
// reads nothing else); Fo and Qs are left unset and the work that feeds only them is dropped.
template <class X, class T, bool FULL = true>
__host__ __device__ inline int gks_flux_pair(const DevParams &P, const int sd, const T q[5], const T g[5][3],
                                             const T n[3], const T dt, T Fo[5], T Fto[5], T Qs[5], T dQs[5]) {
    const T gam = T(P.gamma), K = T(P.K);
    X::pair_shared(true);
    T t1[3];
    if (X::fabs(n[0]) > X::fabs(n[2])) {
        const T r = T(1.0) / X::sqrt(n[0] * n[0] + n[1] * n[1]);
        t1[0] = -n[1] * r; t1[1] = n[0] * r; t1[2] = T(0.0);
    } else {
        const T r = T(1.0) / X::sqrt(n[1] * n[1] + n[2] * n[2]);
        t1[0] = T(0.0); t1[1] = -n[2] * r; t1[2] = n[1] * r;
    }
    const T t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
    const T *fr[3] = {n, t1, t2};
    int err = 0;
    X::pair_shared(false);

    // ---- own side: state and directional derivatives in the face frame -----------------
    T Wk[5], a[3][5];
    Wk[0] = q[0];
    Wk[4] = q[4];
#pragma unroll
    for (int d = 0; d < 3; ++d) Wk[1 + d] = fr[d][0] * q[1] + fr[d][1] * q[2] + fr[d][2] * q[3];
    const T r = Wk[0], ir = T(1.0) / r;
    const T U = Wk[1] * ir, V = Wk[2] * ir, W = Wk[3] * ir;
    const T p = (gam - T(1.0)) * (Wk[4] - T(0.5) * r * (U * U + V * V + W * W));
    if (!(r > T(0.0))) err |= 1;
    if (!(p > T(0.0))) err |= 2;
    const T lm = T(0.5) * r / p, i2lk = p * ir;  // lambda and 1 / (2 lambda)
    const SlopeSolver<T> solk(U, V, W, lm, i2lk, K, T(P.inv_K3));
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        T dv[5], bb[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) dv[v] = fr[dir][0] * g[v][0] + fr[dir][1] * g[v][1] + fr[dir][2] * g[v][2];
        bb[0] = dv[0] * ir;
        bb[4] = dv[4] * ir;
#pragma unroll
        for (int d = 0; d < 3; ++d) bb[1 + d] = (fr[d][0] * dv[1] + fr[d][1] * dv[2] + fr[d][2] * dv[3]) * ir;
        solk.solve(bb, a[dir]);
    }
    T Ak[5], dWk[5];
    {
        MomentsT<T> mf;
        maxwell_moments<X, T>(U, V, W, lm, i2lk, K, 0, mf);
        T S[15], rhs[5] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)};
        psi_matrix<1, 0, 0>(mf, S); sym_mv_acc<X, T>(S, a[0], T(-1.0), rhs);
        psi_matrix<0, 1, 0>(mf, S); sym_mv_acc<X, T>(S, a[1], T(-1.0), rhs);
        psi_matrix<0, 0, 1>(mf, S); sym_mv_acc<X, T>(S, a[2], T(-1.0), rhs);
        solk.solve(rhs, Ak);
#pragma unroll
        for (int v = 0; v < 5; ++v) dWk[v] = r * rhs[v];
    }
    // half-space moment sums of this side: X[0] W0, X[1..3] dW0 per direction, then
    // fh0 <u psi>, fh1 <u psi a.u>, fh2 <u psi A>, wh1 <psi a.u>, wh2 <psi A> (times rho)
    T Xs[9][5];
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int v = 0; v < 5; ++v) Xs[i][v] = T(0.0);
    {
        MomentsT<T> mh;
        maxwell_moments<X, T>(U, V, W, lm, i2lk, K, sd ? -1 : 1, mh);
        T S[15];
        psi_matrix<0, 0, 0>(mh, S);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            Xs[0][v] = r * S[sym_idx(v, 0)];
            Xs[4][v] = r * S[sym_idx(v, 1)];
        }
#pragma unroll
        for (int dir = 0; dir < 3; ++dir) sym_mv_acc<X, T>(S, a[dir], r, Xs[1 + dir]);
        sym_mv_acc<X, T>(S, Ak, r, Xs[8]);
        psi_matrix<1, 0, 0>(mh, S);
        sym_mv_acc<X, T>(S, Ak, r, Xs[6]);
        sym_mv_acc<X, T>(S, a[0], r, Xs[7]);
        psi_matrix<0, 1, 0>(mh, S); sym_mv_acc<X, T>(S, a[1], r, Xs[7]);
        psi_matrix<0, 0, 1>(mh, S); sym_mv_acc<X, T>(S, a[2], r, Xs[7]);
        psi_matrix<2, 0, 0>(mh, S); sym_mv_acc<X, T>(S, a[0], r, Xs[5]);
        psi_matrix<1, 1, 0>(mh, S); sym_mv_acc<X, T>(S, a[1], r, Xs[5]);
        psi_matrix<1, 0, 1>(mh, S); sym_mv_acc<X, T>(S, a[2], r, Xs[5]);
    }
    // pair sums (a + b is order independent, so both lanes hold identical totals)
    X::pair_shared(true);
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int v = 0; v < 5; ++v) Xs[i][v] += X::swap(Xs[i][v]);
    const T p_other = X::swap(p);
    err |= X::swapi(err);

    // ---- equilibrium state at the interface --------------------------------------------
    const T r0 = Xs[0][0], ir0 = T(1.0) / r0;
    const T U0 = Xs[0][1] * ir0, V0 = Xs[0][2] * ir0, Z0 = Xs[0][3] * ir0;
    const T p0 = (gam - T(1.0)) * (Xs[0][4] - T(0.5) * r0 * (U0 * U0 + V0 * V0 + Z0 * Z0));
    if (!(r0 > T(0.0))) err |= 1;
    if (!(p0 > T(0.0))) err |= 2;
    const T lam0 = T(0.5) * r0 / p0, i2l0 = p0 * ir0;  // lambda and 1 / (2 lambda)
    const SlopeSolver<T> sol0(U0, V0, Z0, lam0, i2l0, K, T(P.inv_K3));
    T ab[3][5];
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
        T bb[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) bb[v] = Xs[1 + dir][v] * ir0;
        sol0.solve(bb, ab[dir]);
    }
    // u-moments shifted by sd: psi-moments on the even lane, u psi-moments on the odd lane
    MomentsT<T> m0;
    {
        T us[8];
        line_moments<T>(U0, i2l0, us, 8);
#pragma unroll
        for (int k = 0; k < 7; ++k) m0.u[k] = sd ? us[k + 1] : us[k];
        line_moments<T>(V0, i2l0, m0.v, 6);
        line_moments<T>(Z0, i2l0, m0.w, 6);
        m0.x[0] = T(1.0);
        m0.x[1] = K * i2l0;
        m0.x[2] = K * (K + T(2.0)) * i2l0 * i2l0;
    }
    X::pair_shared(false);
    T e1[5] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)}, e0v[5], e2[5] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)}, Ab[5];
    {
        T S[15];
        psi_matrix<1, 0, 0>(m0, S); sym_mv_acc<X, T>(S, ab[0], T(1.0), e1);
        psi_matrix<0, 1, 0>(m0, S); sym_mv_acc<X, T>(S, ab[1], T(1.0), e1);
        psi_matrix<0, 0, 1>(m0, S); sym_mv_acc<X, T>(S, ab[2], T(1.0), e1);
        // time-derivative coefficient of g0 from the compatibility condition: needs the
        // psi-moment (even lane) version of e1
        T rhs[5];
        X::pair_shared(true);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const T o = X::swap(e1[v]);
            rhs[v] = -(sd ? o : e1[v]);
        }
        sol0.solve(rhs, Ab);
        X::pair_shared(false);
        psi_matrix<0, 0, 0>(m0, S);
#pragma unroll
        for (int v = 0; v < 5; ++v) e0v[v] = S[sym_idx(v, 0)];
        sym_mv_acc<X, T>(S, Ab, T(1.0), e2);
    }
    // collision time (Sec. 5)
    X::pair_shared(true);
    T tau;
    if (P.tau_zero) {
        tau = T(0.0);
    } else {
        const T jump = X::fabs((p - p_other) / (p + p_other));
        tau = P.viscous ? dev_viscosity<X, T>(P, p0 * ir0) / p0 + T(P.tau_C) * jump * dt
                        : (T(P.tau_eps) + T(P.tau_C) * jump) * dt;
    }
    // exp(-dt / tau) = exp(-dt / (2 tau))^2: one exponential serves both windows and the
    // one-sided values below
    const T eh = P.tau_zero ? T(0.0) : X::exp(T(-0.5) * dt / tau), ef = eh * eh;
    T C1[6], C2[6];
    time_integrals<X, T>(dt, tau, ef, P.tau_zero != 0, C1);
    time_integrals<X, T>(T(0.5) * dt, tau, eh, P.tau_zero != 0, C2);
    const T idt = T(1.0) / dt;
    T cn[6], ct[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        if constexpr (FULL) cn[i] = (T(4.0) * C2[i] - C1[i]) * idt;
        ct[i] = T(4.0) * (C1[i] - T(2.0) * C2[i]) * idt * idt;
    }
    X::pair_shared(false);
    // even lane: interface state W^n, W_t^n;  odd lane: flux F^n, F_t^n (face frame)
    T Yn[5], Yt[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const T h0 = sd ? Xs[4][v] : Xs[0][v];
        const T h1 = sd ? Xs[5][v] : Xs[7][v];
        const T h2 = sd ? Xs[6][v] : Xs[8][v];
        if constexpr (FULL)
            Yn[v] = r0 * (cn[0] * e0v[v] + cn[1] * e1[v] + cn[2] * e2[v]) + cn[3] * h0 - cn[4] * h1 - cn[5] * h2;
        Yt[v] = r0 * (ct[0] * e0v[v] + ct[1] * e1[v] + ct[2] * e2[v]) + ct[3] * h0 - ct[4] * h1 - ct[5] * h2;
    }
    T Wn[5], Wt[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        if constexpr (FULL) {
            const T on = X::swap(Yn[v]), ot = X::swap(Yt[v]);
            Wn[v] = sd ? on : Yn[v];
            Wt[v] = sd ? ot : Yt[v];
        } else {
            const T ot = X::swap(Yt[v]);
            Wt[v] = sd ? ot : Yt[v];
        }
    }
    if (P.viscous && P.prandtl_fix && !P.tau_zero) {
        // heat flux relative to the interface velocity, corrected to Pr (odd lane holds F)
        X::pair_shared(true);
        const T uu = U0 * U0 + V0 * V0 + Z0 * Z0, kf = T(1.0 / P.Pr - 1.0);
        const T qt = Yt[4] - (U0 * Yt[1] + V0 * Yt[2] + Z0 * Yt[3]) + T(0.5) * uu * Yt[0] - U0 * Wt[4] +
                     U0 * (U0 * Wt[1] + V0 * Wt[2] + Z0 * Wt[3]) - T(0.5) * U0 * uu * Wt[0];
        if constexpr (FULL) {
            const T qn = Yn[4] - (U0 * Yn[1] + V0 * Yn[2] + Z0 * Yn[3]) + T(0.5) * uu * Yn[0] - U0 * Wn[4] +
                         U0 * (U0 * Wn[1] + V0 * Wn[2] + Z0 * Wn[3]) - T(0.5) * U0 * uu * Wn[0];
            if (sd) {
                Yn[4] += kf * qn;
                Yt[4] += kf * qt;
            }
        } else {
            if (sd) Yt[4] += kf * qt;
        }
        X::pair_shared(false);
    }
    // one-sided interface values (tau0 = tau)
    const T e0 = ef, oe = T(1.0) - e0;
    T Sq[5], St[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        if constexpr (FULL) Sq[v] = oe * Wn[v] + e0 * Wk[v];
        St[v] = oe * Wt[v] + e0 * dWk[v];
    }
    // back to the global frame
    if constexpr (FULL) {
        Qs[0] = Sq[0]; Qs[4] = Sq[4];
    }
    dQs[0] = St[0]; dQs[4] = St[4];
    if constexpr (FULL) {
        Fo[0] = Yn[0]; Fo[4] = Yn[4];
    }
    Fto[0] = Yt[0]; Fto[4] = Yt[4];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if constexpr (FULL) Qs[1 + c] = n[c] * Sq[1] + t1[c] * Sq[2] + t2[c] * Sq[3];
        dQs[1 + c] = n[c] * St[1] + t1[c] * St[2] + t2[c] * St[3];
        // the flux rotation is used from the odd lane only
        X::pair_shared(true);
        if constexpr (FULL) Fo[1 + c] = n[c] * Yn[1] + t1[c] * Yn[2] + t2[c] * Yn[3];
        Fto[1 + c] = n[c] * Yt[1] + t1[c] * Yt[2] + t2[c] * Yt[3];
        X::pair_shared(false);
    }
    bool finite = true;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        if constexpr (FULL)
            finite = finite && X::finite(Fo[v]) && X::finite(Fto[v]) && X::finite(Qs[v]) && X::finite(dQs[v]);
        else
            finite = finite && X::finite(Fto[v]) && X::finite(dQs[v]);
    }
    if (!finite) err |= 4;
    return err;
}

// launch wrappers (cgks_kernels.hip; the flux ones in cgks_flux.hip)
hipError_t launch_metrics(const BlockView &b, const double *nodes, const Metrics &M, long Ntot, int *bad, hipStream_t s);
hipError_t launch_dt(long off, long N, long Ntot, const double *Q, const double *dtm, const DevParams &P,
                     double *part, int nparts, int *flag, hipStream_t s);
hipError_t launch_dt_final(const double *part, int n, double *dt, hipStream_t s);
// Flow diagnostics: part holds nparts * 7 doubles; out 6 doubles (see cgks_diagnostics).
hipError_t launch_diagnostics(long Ntot, const double *Q, const double *G, const double *vol, const DevParams &P,
                              double *part, int nparts, double *out, hipStream_t s);
hipError_t launch_qcriterion(long Ntot, const double *Q, const double *G, double *out, hipStream_t s);
// Diagnostics from the compact reconstruction, one periodic block: coefficients into coef
// (38 doubles per cell and variable, stride Ntot), partial sums into part[nparts][7]; the
// parts of all blocks are then reduced by launch_diagnostics_final into out[6].
hipError_t launch_diagnostics_hq(const BlockView &b, long Ntot, const double *Q, const double *G, const double *L,
                                 const double *nodes, const Metrics &M, const DevConsts *K, const DevParams &P,
                                 double *coef, double *part, int nparts, hipStream_t s);
hipError_t launch_diagnostics_final(const double *part, int nparts, double *out, hipStream_t s);
hipError_t launch_recon(const BlockView &b, long Ntot, const double *Q, const double *G, const double *L,
                        const Metrics &M, const DevConsts *K, const DevParams &P, double *gp, hipStream_t s);
// Per-cell stored matrices (cgks_percell.hip): Rc (34 x 84) and Ec (96 x 34) per cell, tiled by
// the 64 cells of a wave; the buffer holds kPcElems doubles per cell, for ceil(N / 64) * 64 cells.
constexpr int kPcCols = 84;                                 // raw stencil items per variable
constexpr long kPcElems = (long)kNB * kPcCols + 96L * kNB;  // 6120 doubles per cell
constexpr int kPcTile = 64;                                 // cells per storage tile (one wave)
hipError_t launch_percell_setup(const BlockView &b, long Ntot, const Metrics &M, const DevConsts *K, double *pcm,
                                hipStream_t s);
hipError_t launch_recon_percell(const BlockView &b, long Ntot, const double *Q, const double *G, const double *L,
                                const Metrics &M, const DevConsts *K, const DevParams &P, const double *pcm,
                                double *gp, hipStream_t s);
// Inputs and outputs of the blend-weight modes of the matrix-core reconstruction.
struct BlendIO {
    const unsigned char *jump;  // [Ntot] pressure-jump flags (learned weights)
    const unsigned char *mlp;   // packed inference blocks (learned weights)
    double *wexp;               // export: weights used, [Ntot][5][7] (chi, omega_1..6)
    float *xexp;                // export: learned-weight input features, [Ntot][5][18]
};
// Bricks of the staged reconstruction (stg): at most 16 cells in x; the brick with its one-cell
// halo, in rows of kStgRow cells, holds at most kStgCells cells, whose average and gradient of
// one variable (four FP64 planes, 69 KB) sit in LDS beside the 84 KB of constants.
constexpr int kStgRow = 18, kStgCells = 2160;
// the default staged brick: 16 x 8 x 10 cells (80 rows of 16 cells per variable pass)
constexpr int kStgTile[3] = {16, 8, 10};
// workgroup size of the staged reconstruction: 12 waves, 3 per SIMD (one workgroup per CU,
// bound by the LDS; the kernel then fits 168 VGPRs)
constexpr int kStgThreads = 768;
hipError_t launch_recon_mfma(int prec, bool gp32, const WorkList &W, long Ntot, const double *Q, const double *G,
                             const double *L, const Metrics &M, const double *Kblk, const DevParams &P, void *gp,
                             int ngroups, const BlendIO &io, bool exp, bool stg, hipStream_t s);
hipError_t launch_jump(const WorkList &W, long Ntot, const double *Q, const DevParams &P, unsigned char *flag,
                       unsigned long long *count, hipStream_t s);
hipError_t launch_mlp_infer(const float *X, long n, const unsigned char *packed, double *Y, hipStream_t s);
hipError_t launch_mlp_grad(const float *w, const float *X, const float *T, long n, long first, int B, float *S,
                           float *grad, float *loss, hipStream_t s);
hipError_t launch_mlp_adam(float *w, float *m, float *v, const float *g, float lr, float b1, float b2, float eps,
                           int t, hipStream_t s);
int mlp_scratch_floats(int B);
hipError_t launch_gp_export(bool gp32, const BlockView &b, long Ntot, const void *gp, double *out, hipStream_t s);
// Work-list kernels: tiles of at most kFluxTile (flux) or kUpdateTile (update) cells.  The flux
// launches one workgroup per unit (a loop over units would raise its register pressure past
// the 256 VGPRs of two waves per SIMD); the update takes ngroups <= 0 for one workgroup per
// unit, otherwise a persistent grid of ngroups workgroups.
constexpr int kFluxTile = 128, kUpdateTile = 256;
// full = false (second stage) skips the flux and one-sided states, which the second update
// does not read.
// Q: the stage's cell averages (read only with the interface-state limiter, P.positivity).
hipError_t launch_flux(int flux_prec, bool gp32, const WorkList &W, long Ntot, const void *gp, const Metrics &M,
                       const double *dt, const DevParams &P, void *fo, int *flag, bool full, const double *Q,
                       hipStream_t s);
hipError_t launch_flux_points(int flux_prec, long n, const double *ql, const double *gl, const double *qr,
                              const double *gr, const double *nrm, const double *dt, const DevParams &P, double *F,
                              double *Ft, double *S, int *flag, hipStream_t s);
hipError_t launch_update(int stage, bool fo32, const WorkList &W, long Ntot, const void *fo, const Metrics &M,
                         const double *dt, double *Q, double *G, double *L, double *stash, int ngroups,
                         const void *wf, long Wtot, hipStream_t s);
hipError_t launch_flux_wall(int flux_prec, bool gp32, const BlockView &b, int q, long Ntot, const void *gp,
                            const Metrics &M, const double *dt, const DevParams &P, void *fo, void *wf, long Wtot,
                            int *flag, bool full, hipStream_t s);

}  // namespace cgks
