// Compact reconstruction + GENO blend on the matrix cores (v_mfma_f64_16x16x4f64).
//
// On the shared standard cell the reconstruction of every cell and conserved variable is the
// same constant matrix applied to that cell's stacked stencil data (Sec. 4, last paragraph),
// so the work is a dense contraction over all (cell, variable) columns:
//   GEMM1  a  = R b            R: 34 x 72 (eq. compact-big-ref, constrained least squares)
//   GEMMs  zL = L_L^T a,  zT = L_T^T a     IS^L = |zL|^2, IS^tau = |zT|^2 (Cholesky factors
//          of the Gram matrices of the first / second-to-fourth derivatives, Sec. 3.3)
//   GEMM2  y  = E a            E: 96 x 34, point value and reference gradient at the 24 face
//                              Gauss points
// One wavefront owns 16 columns (16 cells of one conserved variable).  Operand layouts of the
// 16x16x4 instructions: lane l supplies A[l%16][l/16] and B[l/16][l%16]; register v of lane l
// receives D[4v + l/16][l%16] (FP64) or D[4(l/16) + v][l%16] (FP32).  Consequences used below:
//   * the stencil item of k-step s and lane group g = l/16 is item perm(4s+g); the k-steps are
//     ordered so that the four lane groups of a step do the same kind of work (no divergence):
//     steps 0..5 face neighbour m (g=0 average difference, g=1..3 reference gradient
//     components), 6..8 edge-neighbour differences (edge 4p+g), 9..14 edge directional
//     derivatives (tau1, tau2 of edge 4p+g), 15..17 line differences (line 4t+g);
//   * GEMM1 leaves one coefficient of a in register v of tile t, which is fed back unchanged as
//     the B operand of the next contractions (their k order is permuted to match on the host);
//   * GEMM2 rows are ordered so that lane group g receives Gauss point g of the tile's face and
//     register v component v (value, d/dxi, d/deta, d/dzeta): blend and back-transform with
//     (J0^T)^-1 stay in the lane.
// The constant blocks are packed on the host in exactly the per-lane order the instruction
// reads and staged once per workgroup in LDS.
#include <hip/hip_runtime.h>

#include "cgks_device.h"
#include "cgks_mlp.h"

namespace cgks {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Arithmetic of the contractions.
//   PrecF64   : FP64 operands, FP64 accumulation (v_mfma_f64_16x16x4f64)
//   PrecF32x3 : split precision on the FP32 matrix cores (v_mfma_f32_16x16x4f32, same operand
//               layout): stencil data b = b_hi + b_lo and constants K = K_hi + K_lo are split
//               into FP32 pairs; K b ~ K_hi b_hi + K_hi b_lo + K_lo b_hi with FP32
//               accumulation.  The follow-up products take the FP32 coefficients as they are:
//               K a ~ K_hi a + K_lo a.
struct PrecF64 {
    using T = double;
    using V = v4d;
    static constexpr int kSplit = 1;
    // k-steps of the coefficient contractions: in this layout k-step 9 holds rows 36..39 of
    // the 34 coefficients only (all zero) and is skipped
    static constexpr int kCoefSteps = 9;
    // coefficients 32 and 33 (the only real rows of the third GEMM1 tile) are accumulated on the
    // vector ALU instead of with 18 mostly-padding matrix instructions
    static constexpr bool kTailOnValu = true;
    // coefficients in parity order (below): block-diagonal smoothness forms, face pairs from
    // one even and one odd product
    static constexpr bool kParity = true;
    using Blend = double;  // type of the blend and Gauss-point output arithmetic
    __device__ static V mma(T a, T b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
struct PrecF32x3 {
    using T = float;
    using V = v4f;
    static constexpr int kCoefSteps = 10;
    static constexpr bool kTailOnValu = false;
    static constexpr bool kParity = false;
    using Blend = float;
    static constexpr int kSplit = 2;
    __device__ static V mma(T a, T b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

// Parity order of the FP64 coefficients.  On the centred standard cell a monomial
// xi^a eta^b zeta^c is even or odd in each axis; the 34 coefficients are ordered by class
// (odd axes) x | y | z | xy | xz | yz | none (9) | xyz (1), so k-step s of the coefficient
// contractions (coefficients 4s..4s+3) holds one class: s = 0..5 the six classes of four, 6
// and 7 eight of the nine even ones, 8 the ninth even one and the odd-odd-odd one.
//   * Products of two basis functions' derivatives of different classes integrate to zero,
//     so the Gram matrices of IS^L and IS^tau are block diagonal and the rows of tile u of their
//     Cholesky-factor products need only k-steps [kISFrom[u], kISTo[u]) (tiles 0..2: L_L^T,
//     3..4: L_T^T over the 31 coefficients of degree >= 2 in the same order).
//   * The Gauss points of the - face of axis q mirror those of the + face, so the - face's
//     values and tangential derivatives are Y_even - Y_odd and its normal derivative
//     Y_odd - Y_even, where Y_even + Y_odd is the + face's and Y_even (Y_odd) takes the
//     coefficients even (odd) in axis q: 10 instead of 18 products per face pair.
constexpr int kISFrom[5] = {0, 4, 8, 0, 4}, kISTo[5] = {4, 9, 9, 5, 9};
constexpr int kParEven[3][6] = {{1, 2, 5, 6, 7, 8}, {0, 2, 4, 6, 7, 8}, {0, 1, 3, 6, 7, 8}};
constexpr int kParOdd[3][4] = {{0, 3, 4, 8}, {1, 3, 5, 8}, {2, 4, 5, 8}};

namespace {

// A lane's cell (index in the mesh) and the index offsets of its six face neighbours on the
// periodic block; an edge neighbour is the sum of two face offsets.  Every index is below
// kMaxCells, so 32-bit integers and 32-bit byte offsets suffice.
struct CellNb {
    int c;
    int dm[3], dp[3];  // offset of the - / + neighbour along x, y, z
};
__device__ inline CellNb cell_nb(const BlockView &b, int ci, int cj, int ck) {
    const int nx = b.nx, nxy = b.nx * b.ny;
    CellNb r;
    r.c = (int)b.off + ci + nx * cj + nxy * ck;
    r.dm[0] = (ci == 0) ? nx - 1 : -1;
    r.dp[0] = (ci == nx - 1) ? 1 - nx : 1;
    r.dm[1] = (cj == 0) ? nxy - nx : -nx;
    r.dp[1] = (cj == b.ny - 1) ? nx - nxy : nx;
    r.dm[2] = (ck == 0) ? (b.nz - 1) * nxy : -nxy;
    r.dp[2] = (ck == b.nz - 1) ? (1 - b.nz) * nxy : nxy;
    return r;
}
// Wall sides the cell (ci, cj, ck) lies on (bit s = 2q + side), with the offsets of gn toward
// them set to zero: the neighbour behind a wall is the mirror image of the cell beside it on the
// inside (the cell itself for a face neighbour).
__device__ inline int wall_touch(const BlockView &b, int ci, int cj, int ck, CellNb &gn) {
    const int w = b.wall;
    int t = 0;
    if ((w & 1) && ci == 0) { t |= 1; gn.dm[0] = 0; }
    if ((w & 2) && ci == b.nx - 1) { t |= 2; gn.dp[0] = 0; }
    if ((w & 4) && cj == 0) { t |= 4; gn.dm[1] = 0; }
    if ((w & 8) && cj == b.ny - 1) { t |= 8; gn.dp[1] = 0; }
    if ((w & 16) && ck == 0) { t |= 16; gn.dm[2] = 0; }
    if ((w & 32) && ck == b.nz - 1) { t |= 32; gn.dp[2] = 0; }
    return t;
}
// Ghost neighbour behind the sides in `crossed`: behind a far-field side the uniform far-field
// state (zero gradient); otherwise the mirror image of its mirror cell's average and physical
// gradient of variable v across the walls (the average changes sign with the variable,
// mirror_sign, the gradient also in its component normal to each wall), continued linearly
// across the non-reflecting sides: the average plus the reference gradient J0^T g of the mirror
// cell nb times the one-cell offset along each such side's axis.
__device__ inline void ghost_mirror(int wall, int crossed, int v, double farv, const double *__restrict__ J0, long Ntot,
                                    int nb, double &q, double g[3]) {
    const int nr = (wall >> 24) & crossed;
#pragma unroll
    for (int s = 0; s < 6; ++s)
        if (((crossed & ~nr) >> s) & 1) {
            const double m = mirror_sign(wall, s, v);
            q *= m;
#pragma unroll
            for (int r = 0; r < 3; ++r) g[r] *= (r == (s >> 1)) ? -m : m;
        }
    if (nr) {
#pragma unroll
        for (int s = 0; s < 6; ++s)
            if ((nr >> s) & 1) {
                const long a = s >> 1;
                const double d = (s & 1) ? 1.0 : -1.0;
                q += d * (J0[a * Ntot + nb] * g[0] + J0[(3 + a) * Ntot + nb] * g[1] + J0[(6 + a) * Ntot + nb] * g[2]);
            }
    }
    const bool far = ((wall >> 16) & crossed) != 0;
    q = far ? farv : q;
#pragma unroll
    for (int r = 0; r < 3; ++r) g[r] = far ? 0.0 : g[r];
}
// Wall sides crossed by gather step st of a lane whose edge signs are (sa, sb).
__device__ inline int step_crossed(int touch, int st, int sa, int sb) {
    if (st < 6) return touch & (1 << st);
    const int p = st - 6, pa = (p < 2) ? 0 : 1, pb = (p == 0) ? 1 : 2;
    return touch & ((1 << (2 * pa + (sa > 0))) | (1 << (2 * pb + (sb > 0))));
}
// Cell read by gather step st (face neighbour st < 6, else edge neighbour of plane st - 6 with
// the lane's edge signs): with the offsets toward wall sides zeroed, the mirror cell.
__device__ inline int step_cell(int c, const CellNb &gn, int st, int sa, int sb) {
    if (st < 6) return c + ((st & 1) ? gn.dp[st >> 1] : gn.dm[st >> 1]);
    const int p = st - 6, pa = (p < 2) ? 0 : 1, pb = (p == 0) ? 1 : 2;
    return c + (sa > 0 ? gn.dp[pa] : gn.dm[pa]) + (sb > 0 ? gn.dp[pb] : gn.dm[pb]);
}

// Cell coordinates of this lane: tile of runs (ty = 0; the wave's first cell is decoded once,
// the lanes step on along x) or brick.  Tail lanes take the last cell of the tile (valid =
// false: they compute a copy and store nothing).
__device__ inline void lane_cell(const Tile &tile, const BlockView &b, int cpr, int chunk, int col, int bx0, int by0,
                                 int bz0, int &ci, int &cj, int &ck, bool &valid) {
    if (tile.ty > 0) {
        const int xo = 16 * (chunk % cpr) + col, row = chunk / cpr;
        valid = xo < tile.count;
        ci = bx0 + (valid ? xo : 0);
        cj = by0 + row % tile.ty;
        ck = bz0 + row / tile.ty;
    } else {
        const unsigned base = (unsigned)tile.start + 16u * (unsigned)chunk;
        const unsigned nx = (unsigned)b.nx, t0 = base / nx;
        valid = 16 * chunk + col < tile.count;
        const int d = valid ? col : tile.count - 1 - 16 * chunk;
        ci = (int)(base - t0 * nx) + d;
        cj = (int)(t0 % (unsigned)b.ny);
        ck = (int)(t0 / (unsigned)b.ny);
        while (ci >= b.nx) {
            ci -= b.nx;
            if (++cj == b.ny) {
                cj = 0;
                ++ck;
            }
        }
    }
}
// element i of a component array (32-bit byte offset from the array's base)
template <class T>
__device__ inline T ld32(const T *base, int i) {
    return *(const T *)((const char *)base + (unsigned)i * (unsigned)sizeof(T));
}

// acc += K * x for an FP64 stencil value x (GEMM1 operand)
template <class PR>
__device__ inline typename PR::V mac_data(const typename PR::T *Ablk, int blk, double x, typename PR::V acc) {
    if constexpr (PR::kSplit == 1) {
        return PR::mma(Ablk[blk * 64], x, acc);
    } else {
        const float xh = (float)x, xl = (float)(x - (double)xh);
        const float kh = Ablk[blk * 64], kl = Ablk[(kMfmaBlocks + blk) * 64];
        acc = PR::mma(kh, xh, acc);
        acc = PR::mma(kh, xl, acc);
        return PR::mma(kl, xh, acc);
    }
}
// acc += K * a for a coefficient a already in the working precision
template <class PR>
__device__ inline typename PR::V mac_coef(const typename PR::T *Ablk, int blk, typename PR::T a, typename PR::V acc) {
    if constexpr (PR::kSplit == 1) {
        return PR::mma(Ablk[blk * 64], a, acc);
    } else {
        acc = PR::mma(Ablk[blk * 64], a, acc);
        return PR::mma(Ablk[(kMfmaBlocks + blk) * 64], a, acc);
    }
}

}  // namespace

// Blend-weight modes: WM = 0 GENO (Sec. 3.3); WM = 1 learned weights (cgks_mlp.h) with GENO
// where the pressure-jump flag of the cell is set.  EXP: also write the weights used
// (wexp [N][5][7]: chi, omega_1..6) and the MLP input features (xexp [N][5][18]).

// STG: the work list holds bricks of at most 16 cells in x (kStgCells bounds the brick with its
// one-cell halo); for each variable in turn the workgroup first copies the brick's averages and
// gradients with the halo into LDS (walls and far-field sides applied there), then every wave
// takes rows of 16 cells and gathers its neighbours from LDS instead of from memory.
template <class PR, class TG, int WM, bool EXP, bool STG = false, int NT = 512>
__global__ void __launch_bounds__(NT) k_recon_mfma(WorkList W, long Ntot, const double *__restrict__ Q,
                                                   const double *__restrict__ G, const double *__restrict__ L,
                                                   Metrics M, const double *__restrict__ Kblk, DevParams P,
                                                   TG *__restrict__ gp, BlendIO io) {
    using T = typename PR::T;
    using V = typename PR::V;
    __shared__ T lds[PR::kSplit * kMfmaBlocks * 64];
    __shared__ double halo[STG ? 4 * kStgCells : 1];  // planes: average, gradient x, y, z
    __shared__ v8bf_t mlp_w[WM ? 3 * 64 : 1];
    __shared__ float mlp_b[WM ? kMlpHidden + 8 : 1];
    for (int i = threadIdx.x; i < kMfmaBlocks * 64; i += blockDim.x) {
        const double k = Kblk[i];
        lds[i] = (T)k;
        if constexpr (PR::kSplit == 2) lds[kMfmaBlocks * 64 + i] = (T)(k - (double)(T)k);
    }
    if constexpr (WM == 1) {
        for (int i = threadIdx.x; i < 3 * 64; i += blockDim.x) mlp_w[i] = ((const v8bf_t *)io.mlp)[i];
        for (int i = threadIdx.x; i < kMlpHidden + 8; i += blockDim.x)
            mlp_b[i] = ((const float *)(io.mlp + kMlpPackBf16 * 2))[i];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    const T *A1 = lds + kMfmaOffA1 * 64 + lane;
    const T *AL = lds + kMfmaOffAL * 64 + lane;
    const T *AT = lds + kMfmaOffAT * 64 + lane;
    const T *A2 = lds + kMfmaOffA2 * 64 + lane;
    // tangential coordinates of this lane's Gauss point (index g on every face)
    const double gq = 0.28867513459481288225;
    const double ta = (g & 1) ? gq : -gq, tb = (g & 2) ? gq : -gq;
    // signs of this lane's edge in the edge steps
    const int sa = (g & 1) ? 1 : -1, sb = (g & 2) ? 1 : -1;

    for (UnitRange ur = unit_range(W.ntiles, W.xcd); ur.u < ur.end; ur.u += ur.step) {
        const Tile tile = W.tiles[ur.u];
        const BlockView b = W.blocks[tile.blk];
        const int cpr = (tile.count + 15) >> 4;  // chunks per run / per brick row
        int bx0 = 0, by0 = 0, bz0 = 0;
        if (tile.ty > 0) {
            bx0 = (int)(tile.start % b.nx);
            const long t0 = tile.start / b.nx;
            by0 = (int)(t0 % b.ny);
            bz0 = (int)(t0 / b.ny);
        }
        const int nit = cpr * (tile.ty > 0 ? tile.ty * tile.tz : 1) * kNV;
        // halo box of a staged brick: x stride kStgRow, rows of HY cells, HY * HZ rows
        const int HY = tile.ty + 2, HZ = tile.tz + 2;
        for (int vp = 0; vp < (STG ? kNV : 1); ++vp) {
        if constexpr (STG) {
            __syncthreads();  // the previous pass has finished reading the halo
            const int nh = kStgRow * HY * HZ;
            const double farv = (vp == 0)   ? P.far[0]
                                : (vp == 1) ? P.far[1]
                                : (vp == 2) ? P.far[2]
                                : (vp == 3) ? P.far[3]
                                            : P.far[4];
            for (int h = threadIdx.x; h < nh; h += blockDim.x) {
                const int hx = h % kStgRow, hr = h / kStgRow;
                if (hx > tile.count + 1) continue;
                int gi = bx0 - 1 + hx, gj = by0 - 1 + hr % HY, gk = bz0 - 1 + hr / HY;
                int crossed = 0;
                // outside the block: periodic image, or the mirror cell inside a wall side
                if (gi < 0) { if (b.wall & 1) { gi = 0; crossed |= 1; } else gi += b.nx; }
                if (gi >= b.nx) { if (b.wall & 2) { gi = b.nx - 1; crossed |= 2; } else gi -= b.nx; }
                if (gj < 0) { if (b.wall & 4) { gj = 0; crossed |= 4; } else gj += b.ny; }
                if (gj >= b.ny) { if (b.wall & 8) { gj = b.ny - 1; crossed |= 8; } else gj -= b.ny; }
                if (gk < 0) { if (b.wall & 16) { gk = 0; crossed |= 16; } else gk += b.nz; }
                if (gk >= b.nz) { if (b.wall & 32) { gk = b.nz - 1; crossed |= 32; } else gk -= b.nz; }
                const int nb = (int)b.off + gi + b.nx * (gj + b.ny * gk);
                double q = ld32(Q + vp * Ntot, nb), gg[3];
    #pragma unroll
                for (int r = 0; r < 3; ++r) gg[r] = ld32(G + (3 * vp + r) * Ntot, nb);
                if (crossed) ghost_mirror(b.wall, crossed, vp, farv, M.J0, Ntot, nb, q, gg);
                halo[h] = q;
    #pragma unroll
                for (int r = 0; r < 3; ++r) halo[(1 + r) * kStgCells + h] = gg[r];
            }
            __syncthreads();
        }
        const int nit_pass = STG ? nit / kNV : nit;
        for (int it = __builtin_amdgcn_readfirstlane(wave); it < nit_pass; it += nwaves) {
            const int v = STG ? vp : it % kNV;
            const int chunk = STG ? it : it / kNV;
            bool valid;
            int ci, cj, ck;
            lane_cell(tile, b, cpr, chunk, col, bx0, by0, bz0, ci, cj, ck, valid);
            const CellNb cn = cell_nb(b, ci, cj, ck);
            const int c = cn.c;
            const double *Qv = Q + v * Ntot;
            const double *Gv = G + 3 * v * Ntot;
            const double *Lv = L + 12 * v * Ntot;
            double J0[3][3];
    #pragma unroll
            for (int r = 0; r < 3; ++r)
    #pragma unroll
                for (int s = 0; s < 3; ++s) J0[r][s] = ld32(M.J0 + (3 * r + s) * Ntot, c);
            const double q0 = ld32(Qv, c);

            V acc[3] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
            double a32 = 0.0, a33 = 0.0;  // partial sums of coefficients 32, 33 (kTailOnValu)
            // GEMM1 step: the stencil item of this lane times column sb of R
            auto gemm1 = [&](int sb, double item) {
                acc[0] = mac_data<PR>(A1, sb, item, acc[0]);
                acc[1] = mac_data<PR>(A1, 18 + sb, item, acc[1]);
                if constexpr (PR::kTailOnValu) {
                    const T *r2 = lds + (kMfmaOffA1 + 36 + sb) * 64 + 16 * g;  // rows 32, 33 of tile 2
                    a32 = fma((double)r2[0], item, a32);
                    a33 = fma((double)r2[1], item, a33);
                } else {
                    acc[2] = mac_data<PR>(A1, 36 + sb, item, acc[2]);
                }
            };
            // line derivatives of the cell (steps 15..17), loaded ahead of the neighbour gather
            double lval[3];
    #pragma unroll
            for (int s = 0; s < 3; ++s) lval[s] = ld32(Lv + 4 * s * Ntot, g * (int)Ntot + c);
            // ---- steps 0..14: face neighbours m (steps m), then edge neighbours 4p+g (steps
            // 6+p, 9+2p, 10+2p).  The average and gradient of all nine neighbours a lane needs are
            // requested before the first contraction, so the wave waits for memory once.
            // ghost neighbours behind wall sides: their mirror cells, mirrored below.  Periodic
            // blocks never take the mirror branch; the kernel keeps one form for both because
            // this one, which completes the gather before the first contraction, measured faster
            // (32.5 against 33.5 ms per FP64 launch at 256^3, bitwise equal results).
            CellNb gn = cn;
            const int touch = wall_touch(b, ci, cj, ck, gn);
            // far-field value of this wave's variable (wave-uniform selects, no indexed access)
            const double farv = (v == 0)   ? P.far[0]
                                : (v == 1) ? P.far[1]
                                : (v == 2) ? P.far[2]
                                : (v == 3) ? P.far[3]
                                           : P.far[4];
            double nq[9], ng[9][3];
            // staged: this lane's cell in the halo box and the box offset of each gather step;
            // the steps read LDS one at a time below (short latency: no registers held for all
            // nine neighbours)
            const int hb = STG ? (ci - bx0 + 1) + kStgRow * ((cj - by0 + 1) + HY * (ck - bz0 + 1)) : 0;
            auto halo_at = [&](int st) {
                const int hs[3] = {1, kStgRow, kStgRow * HY};
                if (st < 6) return hb + ((st & 1) ? hs[st >> 1] : -hs[st >> 1]);
                const int p = st - 6, pa = (p < 2) ? 0 : 1, pb = (p == 0) ? 1 : 2;
                return hb + sa * hs[pa] + sb * hs[pb];
            };
            if constexpr (STG) {
                (void)touch;
                (void)farv;
            } else {
    #pragma unroll
                for (int st = 0; st < 9; ++st) {
                    int nb;
                    if (st < 6) {
                        nb = c + ((st & 1) ? gn.dp[st >> 1] : gn.dm[st >> 1]);
                    } else {
                        const int p = st - 6, pa = (p < 2) ? 0 : 1, pb = (p == 0) ? 1 : 2;
                        nb = c + (sa > 0 ? gn.dp[pa] : gn.dm[pa]) + (sb > 0 ? gn.dp[pb] : gn.dm[pb]);
                    }
                    nq[st] = ld32(Qv, nb);
                    ng[st][0] = ld32(Gv, nb);
                    ng[st][1] = ld32(Gv + Ntot, nb);
                    ng[st][2] = ld32(Gv + 2 * Ntot, nb);
                }
    #pragma unroll
                for (int st = 0; st < 9; ++st) {
                    const int crossed = step_crossed(touch, st, sa, sb);
                    if (crossed) ghost_mirror(b.wall, crossed, v, farv, M.J0, Ntot, step_cell(c, gn, st, sa, sb), nq[st],
                                              ng[st]);
                }
            }
    #pragma unroll
            for (int st = 0; st < 9; ++st) {
                if constexpr (STG) {
                    const int h = halo_at(st);
                    nq[st] = halo[h];
                    ng[st][0] = halo[kStgCells + h];
                    ng[st][1] = halo[2 * kStgCells + h];
                    ng[st][2] = halo[3 * kStgCells + h];
                }
                const double d = nq[st] - q0;
                double rg[3];
    #pragma unroll
                for (int r = 0; r < 3; ++r) rg[r] = J0[0][r] * ng[st][0] + J0[1][r] * ng[st][1] + J0[2][r] * ng[st][2];
                if (st < 6) {
                    const double item = (g == 0) ? d : (g == 1) ? rg[0] : (g == 2) ? rg[1] : rg[2];
                    gemm1(st, item);
                } else {
                    const int p = st - 6;
                    const int pa = (p < 2) ? 0 : 1, pb = (p == 0) ? 1 : 2, pc = 3 - pa - pb;
                    const double e1 = (pc == 0) ? rg[0] : (pc == 1) ? rg[1] : rg[2];
                    const double ra = (pa == 0) ? rg[0] : rg[1], rb = (pb == 1) ? rg[1] : rg[2];
                    const double e2 = (sa * ra + sb * rb) * 0.70710678118654752440;
                    gemm1(6 + p, d);
                    gemm1(9 + 2 * p, e1);
                    gemm1(10 + 2 * p, e2);
                }
                __builtin_amdgcn_sched_barrier(0);  // keep each step's operand loads with its step
            }
            // ---- steps 15..17: line differences 4t+g ---------------------------------------------
            double lsum[3];
    #pragma unroll
            for (int s = 0; s < 3; ++s) {
                const double ln = lval[s];
                gemm1(15 + s, ln);
                double x = ln + __shfl_xor(ln, 16, 64);
                lsum[s] = x + __shfl_xor(x, 32, 64);
            }
            if constexpr (PR::kTailOnValu) {
                // sum over the four lane groups; in register 0 of tile 2, lane group g holds row 32+g
                a32 += __shfl_xor(a32, 16, 64);
                a32 += __shfl_xor(a32, 32, 64);
                a33 += __shfl_xor(a33, 16, 64);
                a33 += __shfl_xor(a33, 32, 64);
                acc[2] = V{(g == 0) ? a32 : ((g == 1) ? a33 : 0.0), 0.0, 0.0, 0.0};
            }

            // back-transform of the Gauss-point gradients, requested here so that the smoothness forms
            // and weights below cover its latency
            typename PR::Blend JiT[3][3];
    #pragma unroll
            for (int r = 0; r < 3; ++r)
    #pragma unroll
                for (int s = 0; s < 3; ++s) JiT[r][s] = ld32(M.JiT + (3 * r + s) * Ntot, c);

            // ---- blend weights ------------------------------------------------------------------------
            // FP64 reconstruction: all in FP64.  FP32x3: the blend and the Gauss-point outputs run in
            // FP32 (the stored values are FP32 and the split products carry 2^-24 of the data).
            using RW = typename PR::Blend;
            RW chi = 1, bbar[3] = {0, 0, 0};
            if (!P.linear) {
                // linear sub-polynomials of the six face sub-stencils (eq. compact-sub-2)
                const RW lm[3] = {RW(0.25 * lsum[0]), RW(0.25 * lsum[1]), RW(0.25 * lsum[2])};
                RW fdiff[6];  // face-neighbour differences: the averages gathered in steps 0..5
    #pragma unroll
                for (int m = 0; m < 6; ++m) fdiff[m] = RW((STG ? halo[halo_at(m)] : nq[m]) - q0);
                // learned-weight inputs: differences and line derivatives over their largest magnitude
                double fscale = 1.0;
                if constexpr (WM == 1 || EXP) {
                    double mx = fmax(fmax(fabs(lval[0]), fabs(lval[1])), fabs(lval[2]));
                    mx = fmax(mx, __shfl_xor(mx, 16, 64));
                    mx = fmax(mx, __shfl_xor(mx, 32, 64));
    #pragma unroll
                    for (int m = 0; m < 6; ++m) mx = fmax(mx, fabs(fdiff[m]));
                    fscale = 1.0 / (mx + 1e-12);
                }
                double chi_l = 1.0, om_l[6] = {0, 0, 0, 0, 0, 0};
                bool geno = true;
                if constexpr (WM == 1) {
                    geno = io.jump[c] != 0;
                    v8bf_t xin;
    #pragma unroll
                    for (int jx = 0; jx < 8; ++jx) {
                        const double f = (jx < 3) ? lval[jx]
                                                  : ((jx < 5 && g < 3) ? fdiff[2 * g + jx - 3] : 0.0);
                        xin[jx] = (__bf16)(float)(f * fscale);
                    }
                    float z[7];
                    mlp_eval(mlp_w + lane, mlp_b, mlp_b + kMlpHidden, xin, g, col, z);
                    mlp_weights(z, chi_l, om_l);
                }
                RW chi_g = 1, om_g[6] = {0, 0, 0, 0, 0, 0};
                if (WM == 0 || __any(geno)) {
                    // path function chi: IS^L and IS^tau from the Cholesky-factor contractions
                    RW isl = 0, ist = 0;
    #pragma unroll
                    for (int u = 0; u < 5; ++u) {  // tiles 0..2: L_L^T rows, tiles 3..4: L_T^T rows
                        const int base = (u < 3) ? kMfmaOffAL + u * 10 : kMfmaOffAT + (u - 3) * 10;
                        // the Cholesky factors are triangular: rows 16w.. of tile w = u (mod 3) vanish on
                        // the coefficients of k-steps below 4w, which are skipped (their products are
                        // zero); in parity order they are also block diagonal
                        const int s0 = PR::kParity ? kISFrom[u] : 4 * ((u < 3) ? u : u - 3);
                        const int s1 = PR::kParity ? kISTo[u] : PR::kCoefSteps;
                        V z = {0, 0, 0, 0};
    #pragma unroll
                        for (int s = 0; s < PR::kCoefSteps; ++s)
                            if (s >= s0 && s < s1) z = mac_coef<PR>(lds + lane, base + s, acc[s >> 2][s & 3], z);
                        const RW zz = (RW)z[0] * z[0] + (RW)z[1] * z[1] + (RW)z[2] * z[2] + (RW)z[3] * z[3];
                        if (u < 3) isl += zz;
                        else ist += zz;
                    }
                    isl += __shfl_xor(isl, 16, 64);
                    isl += __shfl_xor(isl, 32, 64);
                    ist += __shfl_xor(ist, 16, 64);
                    ist += __shfl_xor(ist, 32, 64);
                    const RW eps = RW(P.geno_eps);
                    const RW ish = isl + ist;
                    const RW rh = ist / (ish + eps), rl = ist / (isl + eps);
                    RW ah, al;
                    if (P.geno_r == 2.0) {
                        ah = RW(1) + rh * rh;
                        al = RW(1) + rl * rl;
                    } else {
                        ah = RW(1) + pow(rh, RW(P.geno_r));
                        al = RW(1) + pow(rl, RW(P.geno_r));
                    }
                    // tanh(x) rounds to 1 once 2 exp(-2x) is below half an ulp of 1 (x > 19.1 in FP64,
                    // x > 9.1 in FP32); the library call runs only if some lane of the wave is below
                    const RW x = RW(P.geno_C) * (RW(2) * ah / (ah + al));
                    const RW x_one = (sizeof(RW) == 8) ? RW(20) : RW(10);
                    RW th = RW(1);
                    if (__any(x <= x_one)) th = (x > x_one) ? RW(1) : tanh(x);
                    chi_g = th * RW(P.inv_tanhC);
                    // the linear weights enter only through (1 - chi); a wave whose cells all have
                    // chi = 1 skips them (they are always formed when exported)
                    if (EXP || __any(geno && chi_g != RW(1))) {
                        if constexpr (sizeof(RW) == 8) {
                            double wsum = 0.0;
            #pragma unroll
                            for (int m = 0; m < 6; ++m) {
                                const int q = m >> 1;
                                const double bn = (m & 1) ? fdiff[m] : -fdiff[m];
                                double is = eps + bn * bn;
            #pragma unroll
                                for (int t = 0; t < 3; ++t)
                                    if (t != q) is += lm[t] * lm[t];
                                const double is2 = is * is;
                                om_g[m] = (1.0 / 6.0) / (is2 * is2 * is);
                                wsum += om_g[m];
                            }
                            const double iw = 1.0 / wsum;
            #pragma unroll
                            for (int m = 0; m < 6; ++m) om_g[m] *= iw;
                        } else {
                            // (1/6)/IS_m^5 normalised by the largest 1/IS_m (FP32 range)
                            RW tmax = 0;
        #pragma unroll
                            for (int m = 0; m < 6; ++m) {
                                const int q = m >> 1;
                                RW is = eps + fdiff[m] * fdiff[m];
        #pragma unroll
                                for (int t = 0; t < 3; ++t)
                                    if (t != q) is += lm[t] * lm[t];
                                om_g[m] = RW(1) / is;
                                tmax = fmax(tmax, om_g[m]);
                            }
                            RW wsum = 0;
        #pragma unroll
                            for (int m = 0; m < 6; ++m) {
                                const RW r = om_g[m] / tmax, r2 = r * r;
                                om_g[m] = r2 * r2 * r;
                                wsum += om_g[m];
                            }
                            const RW iw = RW(1) / wsum;
        #pragma unroll
                            for (int m = 0; m < 6; ++m) om_g[m] *= iw;
                        }
                    }
                }
                chi = geno ? chi_g : RW(chi_l);
    #pragma unroll
                for (int m = 0; m < 6; ++m) {
                    const int q = m >> 1;
                    const RW w = geno ? om_g[m] : RW(om_l[m]);
                    const RW bn = (m & 1) ? fdiff[m] : -fdiff[m];
    #pragma unroll
                    for (int t = 0; t < 3; ++t) bbar[t] += w * ((t == q) ? bn : lm[t]);
                }
                if constexpr (EXP) {
                    if (valid) {
                        const long sidx = (long)c * kNV + v;
                        if (g == 0) {
                            io.wexp[sidx * 7] = chi;
    #pragma unroll
                            for (int m = 0; m < 6; ++m) io.wexp[sidx * 7 + 1 + m] = geno ? om_g[m] : om_l[m];
                        }
    #pragma unroll
                        for (int jx = 0; jx < 5; ++jx) {
                            const int f = mlp_slot_feature(g, jx);
                            if (f >= 0) {
                                const double val = (jx < 3) ? lval[jx] : fdiff[2 * g + jx - 3];
                                io.xexp[sidx * kMlpIn + f] = (float)(val * fscale);
                            }
                        }
                    }
                }
            }
            const RW om = RW(1) - chi;

            // ---- Gauss-point values: face m = tile u, Gauss point k = g ----------------------------
            // the cell in the Gauss-point buffer (rows padded to nxp cells)
            const int gl = c - (int)b.off;
            const int gc = (int)b.goff + gl + ((b.nxp == b.nx) ? 0 : (b.nxp - b.nx) * (gl / b.nx));
            auto emit = [&](int u, const V y) __attribute__((always_inline)) {
                const int q = u >> 1;
                const RW xq = (u & 1) ? RW(0.5) : RW(-0.5);
                const RW x0 = (q == 0) ? xq : RW(ta);
                const RW x1 = (q == 1) ? xq : ((q == 0) ? RW(ta) : RW(tb));
                const RW x2 = (q == 2) ? xq : RW(tb);
                double val;
                if constexpr (sizeof(RW) == 8)
                    val = q0 + chi * (double)y[0] + om * (bbar[0] * x0 + bbar[1] * x1 + bbar[2] * x2);
                else  // deviation from the cell average in FP32, added to the FP64 average
                    val = q0 + (double)(chi * (RW)y[0] + om * (bbar[0] * x0 + bbar[1] * x1 + bbar[2] * x2));
                const RW r0 = chi * (RW)y[1] + om * bbar[0], r1 = chi * (RW)y[2] + om * bbar[1],
                         r2 = chi * (RW)y[3] + om * bbar[2];
                // face u is the + face of this cell (side 0) or the + face of the - neighbour (side 1)
                const int side = (u & 1) ? 0 : 1;
                // face record in the Gauss-point buffer: this cell's (+ face) or the minus
                // neighbour's, periodic in the block (its offset from the cell's sign of cn.dm)
                const int f = (u & 1) ? gc
                                      : gc + ((q == 0)   ? cn.dm[0]
                                              : (q == 1) ? ((cn.dm[1] < 0) ? -b.nxp : (b.ny - 1) * b.nxp)
                                                         : ((cn.dm[2] < 0) ? -b.ny * b.nxp : (b.nz - 1) * b.ny * b.nxp));
                if (valid) {
                    const long gs = b.gstride;
                    TG *dst = gp + ((long)(((q * 2 + side) * 4 + g) * 20 + v * 4)) * gs + f;
                    __builtin_nontemporal_store((TG)val, dst);
                    __builtin_nontemporal_store((TG)(JiT[0][0] * r0 + JiT[0][1] * r1 + JiT[0][2] * r2), dst + gs);
                    __builtin_nontemporal_store((TG)(JiT[1][0] * r0 + JiT[1][1] * r1 + JiT[1][2] * r2), dst + 2 * gs);
                    __builtin_nontemporal_store((TG)(JiT[2][0] * r0 + JiT[2][1] * r1 + JiT[2][2] * r2), dst + 3 * gs);
                }
            };
            if constexpr (PR::kParity) {
    #pragma unroll
                for (int q = 0; q < 3; ++q) {
                    V ye = {0, 0, 0, 0}, yo = {0, 0, 0, 0};
    #pragma unroll
                    for (int j = 0; j < 6; ++j) {
                        const int st = kParEven[q][j];
                        ye = mac_coef<PR>(lds + lane, kMfmaOffA2 + q * 10 + j, acc[st >> 2][st & 3], ye);
                    }
    #pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int st = kParOdd[q][j];
                        yo = mac_coef<PR>(lds + lane, kMfmaOffA2 + q * 10 + 6 + j, acc[st >> 2][st & 3], yo);
                    }
                    V yp, ym;
    #pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        yp[r] = ye[r] + yo[r];
                        ym[r] = (r == 1 + q) ? yo[r] - ye[r] : ye[r] - yo[r];
                    }
                    emit(2 * q, ym);
                    emit(2 * q + 1, yp);
                    __builtin_amdgcn_sched_barrier(0);  // one face pair at a time (register pressure)
                }
            } else {
    #pragma unroll
                for (int u = 0; u < 6; ++u) {
                    V y = {0, 0, 0, 0};
    #pragma unroll
                    for (int s = 0; s < PR::kCoefSteps; ++s)
                        y = mac_coef<PR>(lds + lane, kMfmaOffA2 + u * 10 + s, acc[s >> 2][s & 3], y);
                    emit(u, y);
                }
            }
        }
        }  // variable passes of a staged brick
    }
}

// ------------------------------------------------------------------------------------------
// BF16x3 variant on the 16x16x32 BF16 matrix cores (gfx950).  Lane l supplies A[l%16][8(l/16)+j]
// and B[8(l/16)+j][l%16], j = 0..7, and register v receives D[4(l/16)+v][l%16] (FP32).  The 18
// stencil slots of the 16x16x4 kernels are packed as slot 8s + j of k-step s (slots 18..23
// zero); the 12 coefficients a lane holds after GEMM1 are packed the same way for the
// follow-up products.  Every product is split: x = x_hi + x_lo and K = K_hi + K_lo in BF16,
// K x ~ K_hi x_hi + K_hi x_lo + K_lo x_hi, FP32 accumulation.
// ------------------------------------------------------------------------------------------
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

namespace {
// Store x as the BF16 pair (hi, lo) in slot sl of the k-step vectors h[sl/8], l[sl/8].
__device__ inline void put_bf16(v8bf *h, v8bf *l, int sl, double x) {
    const __bf16 hi = (__bf16)(float)x;
    h[sl / 8][sl % 8] = hi;
    l[sl / 8][sl % 8] = (__bf16)(float)(x - (double)(float)hi);
}
// Store x as the BF16 pair (hi, lo) in slot sl, from an FP32 value.
__device__ inline void put_bf16f(v8bf *h, v8bf *l, int sl, float x) {
    const __bf16 hi = (__bf16)x;
    h[sl / 8][sl % 8] = hi;
    l[sl / 8][sl % 8] = (__bf16)(x - (float)hi);
}
__device__ inline v4f mma3(const v8bf *Kb, int blk, const v8bf &xh, const v8bf &xl, v4f acc) {
    const v8bf kh = Kb[blk * 64], kl = Kb[(kBfBlocks + blk) * 64];
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, xh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, xl, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(kl, xh, acc, 0, 0, 0);
}
}  // namespace

template <class TG>
__global__ void __launch_bounds__(512) k_recon_bf16(WorkList W, long Ntot, const double *__restrict__ Q,
                                                    const double *__restrict__ G, const double *__restrict__ L,
                                                    Metrics M, const double *__restrict__ Kbf, DevParams P,
                                                    TG *__restrict__ gp) {
    __shared__ v8bf lds[2 * kBfBlocks * 64];
    for (int i = threadIdx.x; i < kBfBlocks * 64; i += blockDim.x) {
        v8bf h, lo;
#pragma unroll
        for (int j = 0; j < 8; ++j) put_bf16(&h, &lo, j, Kbf[i * 8 + j]);
        lds[i] = h;
        lds[kBfBlocks * 64 + i] = lo;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    const v8bf *Kb = lds + lane;
    const double gq = 0.28867513459481288225;
    const double ta = (g & 1) ? gq : -gq, tb = (g & 2) ? gq : -gq;
    const int sa = (g & 1) ? 1 : -1, sb = (g & 2) ? 1 : -1;

    for (UnitRange ur = unit_range(W.ntiles, W.xcd); ur.u < ur.end; ur.u += ur.step) {
        const Tile tile = W.tiles[ur.u];
        const BlockView b = W.blocks[tile.blk];
        const int cpr = (tile.count + 15) >> 4;  // chunks per run / per brick row
        int bx0 = 0, by0 = 0, bz0 = 0;
        if (tile.ty > 0) {
            bx0 = (int)(tile.start % b.nx);
            const long t0 = tile.start / b.nx;
            by0 = (int)(t0 % b.ny);
            bz0 = (int)(t0 / b.ny);
        }
        const int nit = cpr * (tile.ty > 0 ? tile.ty * tile.tz : 1) * kNV;
        for (int it = __builtin_amdgcn_readfirstlane(wave); it < nit; it += nwaves) {
            const int v = it % kNV;
            const int chunk = it / kNV;
            bool valid;
            int ci, cj, ck;
            lane_cell(tile, b, cpr, chunk, col, bx0, by0, bz0, ci, cj, ck, valid);
            const CellNb cn = cell_nb(b, ci, cj, ck);
            const int c = cn.c;
            const double *Qv = Q + v * Ntot;
            const double *Gv = G + 3 * v * Ntot;
            const double *Lv = L + 12 * v * Ntot;
            // The split products carry 2^-17 of their operands, so the vector work here runs in
            // FP32 (2^-24); only the differences to the cell average are formed in FP64.
            double J0d[3][3];
    #pragma unroll
            for (int r = 0; r < 3; ++r)
    #pragma unroll
                for (int s = 0; s < 3; ++s) J0d[r][s] = ld32(M.J0 + (3 * r + s) * Ntot, c);
            const double q0 = ld32(Qv, c);

            // ---- the 18 stencil slots of this lane, split into BF16 hi/lo, slot 8s + j ----------
            v8bf bh[3], bl[3];
    #pragma unroll
            for (int s = 0; s < 3; ++s)
    #pragma unroll
                for (int j = 0; j < 8; ++j) {
                    bh[s][j] = (__bf16)0.0f;
                    bl[s][j] = (__bf16)0.0f;
                }
            // all nine neighbours first (one wait for memory), then the slots
            // ghost neighbours behind wall sides: their mirror cells, mirrored below.  Periodic
            // blocks never take the mirror branch; the kernel keeps one form for both because
            // this one, which completes the gather before the first contraction, measured faster
            // (32.5 against 33.5 ms per FP64 launch at 256^3, bitwise equal results).
            CellNb gn = cn;
            const int touch = wall_touch(b, ci, cj, ck, gn);
            // far-field value of this wave's variable (wave-uniform selects, no indexed access)
            const double farv = (v == 0)   ? P.far[0]
                                : (v == 1) ? P.far[1]
                                : (v == 2) ? P.far[2]
                                : (v == 3) ? P.far[3]
                                           : P.far[4];
            double nq[9], ng[9][3];
    #pragma unroll
            for (int st = 0; st < 9; ++st) {
                int nb;
                if (st < 6) {
                    nb = c + ((st & 1) ? gn.dp[st >> 1] : gn.dm[st >> 1]);
                } else {
                    const int p = st - 6, pa = (p < 2) ? 0 : 1, pb = (p == 0) ? 1 : 2;
                    nb = c + (sa > 0 ? gn.dp[pa] : gn.dm[pa]) + (sb > 0 ? gn.dp[pb] : gn.dm[pb]);
                }
                nq[st] = ld32(Qv, nb);
                ng[st][0] = ld32(Gv, nb);
                ng[st][1] = ld32(Gv + Ntot, nb);
                ng[st][2] = ld32(Gv + 2 * Ntot, nb);
            }
    #pragma unroll
            for (int st = 0; st < 9; ++st) {
                const int crossed = step_crossed(touch, st, sa, sb);
                if (crossed) ghost_mirror(b.wall, crossed, v, farv, M.J0, Ntot, step_cell(c, gn, st, sa, sb), nq[st], ng[st]);
            }
            double lvd[3];
    #pragma unroll
            for (int s = 0; s < 3; ++s) lvd[s] = ld32(Lv + 4 * s * Ntot, g * (int)Ntot + c);
            __builtin_amdgcn_sched_barrier(0);  // every request above is in flight before the first use
            const float lv[3] = {(float)lvd[0], (float)lvd[1], (float)lvd[2]};
            float J0[3][3];
    #pragma unroll
            for (int r = 0; r < 3; ++r)
    #pragma unroll
                for (int s = 0; s < 3; ++s) J0[r][s] = (float)J0d[r][s];
            float fdiff[6];
    #pragma unroll
            for (int m = 0; m < 6; ++m) {
                const float g0 = (float)ng[m][0], g1 = (float)ng[m][1], g2 = (float)ng[m][2];
                fdiff[m] = (float)(nq[m] - q0);
                const float r0 = J0[0][0] * g0 + J0[1][0] * g1 + J0[2][0] * g2;
                const float r1 = J0[0][1] * g0 + J0[1][1] * g1 + J0[2][1] * g2;
                const float r2 = J0[0][2] * g0 + J0[1][2] * g1 + J0[2][2] * g2;
                put_bf16f(bh, bl, m, (g == 0) ? fdiff[m] : (g == 1) ? r0 : (g == 2) ? r1 : r2);
            }
    #pragma unroll
            for (int p = 0; p < 3; ++p) {
                const int pa = (p < 2) ? 0 : 1, pb = (p == 0) ? 1 : 2, pc = 3 - pa - pb;
                const int s0 = 6 + p, s1 = 9 + 2 * p, s2 = 10 + 2 * p;
                put_bf16f(bh, bl, s0, (float)(nq[6 + p] - q0));
                const float g0 = (float)ng[6 + p][0], g1 = (float)ng[6 + p][1], g2 = (float)ng[6 + p][2];
                float rg[3];
    #pragma unroll
                for (int s = 0; s < 3; ++s) rg[s] = J0[0][s] * g0 + J0[1][s] * g1 + J0[2][s] * g2;
                put_bf16f(bh, bl, s1, rg[pc]);
                put_bf16f(bh, bl, s2, ((float)sa * rg[pa] + (float)sb * rg[pb]) * 0.70710678118654752440f);
            }
            float lsum[3];
    #pragma unroll
            for (int s = 0; s < 3; ++s) {
                const float ln = lv[s];
                put_bf16f(bh, bl, 15 + s, ln);
                const float x = ln + __shfl_xor(ln, 16, 64);
                lsum[s] = x + __shfl_xor(x, 32, 64);
            }
            // ---- GEMM1: a = R b ---------------------------------------------------------------------
            v4f acc[3] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    #pragma unroll
            for (int t = 0; t < 3; ++t)
    #pragma unroll
                for (int s = 0; s < 3; ++s) acc[t] = mma3(Kb, kBfOffA1 + t * 3 + s, bh[s], bl[s], acc[t]);
            // coefficients of this lane as BF16 hi/lo, slot 8s' + j = 4t + v
            v8bf ch[2], cl2[2];
    #pragma unroll
            for (int s = 0; s < 2; ++s)
    #pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int sig = 8 * s + j;
                    const float x = (sig < 12) ? acc[sig / 4][sig % 4] : 0.0f;
                    const __bf16 h = (__bf16)x;
                    ch[s][j] = h;
                    cl2[s][j] = (__bf16)(x - (float)h);
                }

            // back-transform of the Gauss-point gradients, requested before the smoothness forms
            double JiTd[3][3];
    #pragma unroll
            for (int r = 0; r < 3; ++r)
    #pragma unroll
                for (int s = 0; s < 3; ++s) JiTd[r][s] = ld32(M.JiT + (3 * r + s) * Ntot, c);
            float chi = 1.0f, bbar[3] = {0.0f, 0.0f, 0.0f};
            if (!P.linear) {
                float isl = 0.0f, ist = 0.0f;
    #pragma unroll
                for (int u = 0; u < 5; ++u) {
                    const int base = (u < 3) ? kBfOffAL + u * 2 : kBfOffAT + (u - 3) * 2;
                    v4f z = {0, 0, 0, 0};
    #pragma unroll
                    for (int s = 0; s < 2; ++s) z = mma3(Kb, base + s, ch[s], cl2[s], z);
                    const float zz = z[0] * z[0] + z[1] * z[1] + z[2] * z[2] + z[3] * z[3];
                    if (u < 3) isl += zz;
                    else ist += zz;
                }
                isl += __shfl_xor(isl, 16, 64);
                isl += __shfl_xor(isl, 32, 64);
                ist += __shfl_xor(ist, 16, 64);
                ist += __shfl_xor(ist, 32, 64);
                const float eps = (float)P.geno_eps;
                const float ish = isl + ist;
                const float rh = ist / (ish + eps), rl = ist / (isl + eps);
                float ah, al;
                if (P.geno_r == 2.0) {
                    ah = 1.0f + rh * rh;
                    al = 1.0f + rl * rl;
                } else {
                    ah = 1.0f + powf(rh, (float)P.geno_r);
                    al = 1.0f + powf(rl, (float)P.geno_r);
                }
                // tanhf(x) rounds to 1 for x > 9.1; the library call runs only if a lane is below 10
                const float x = (float)P.geno_C * (2.0f * ah / (ah + al));
                float th = 1.0f;
                if (__any(x <= 10.0f)) th = (x > 10.0f) ? 1.0f : tanhf(x);
                chi = th * (float)P.inv_tanhC;
                // linear weights (1/6)/IS_m^5, normalised by the largest 1/IS_m so that the fifth
                // powers stay inside the FP32 range; they enter only through (1 - chi)
                const float lm[3] = {0.25f * lsum[0], 0.25f * lsum[1], 0.25f * lsum[2]};
                if (__any(chi != 1.0f)) {
                    float ti[6], tmax = 0.0f;
        #pragma unroll
                    for (int m = 0; m < 6; ++m) {
                        const int q = m >> 1;
                        const float bn = fdiff[m];
                        float is = eps + bn * bn;
        #pragma unroll
                        for (int t = 0; t < 3; ++t)
                            if (t != q) is += lm[t] * lm[t];
                        ti[m] = 1.0f / is;
                        tmax = fmaxf(tmax, ti[m]);
                    }
                    float wsum = 0.0f;
        #pragma unroll
                    for (int m = 0; m < 6; ++m) {
                        const float r = ti[m] / tmax, r2 = r * r;
                        ti[m] = r2 * r2 * r;
                        wsum += ti[m];
                    }
                    const float iw = 1.0f / wsum;
        #pragma unroll
                    for (int m = 0; m < 6; ++m) {
                        const int q = m >> 1;
                        const float w = ti[m] * iw;
                        const float bn = (m & 1) ? fdiff[m] : -fdiff[m];
        #pragma unroll
                        for (int t = 0; t < 3; ++t) bbar[t] += w * ((t == q) ? bn : lm[t]);
                    }
                }
            }
            float JiT[3][3];
    #pragma unroll
            for (int r = 0; r < 3; ++r)
    #pragma unroll
                for (int s = 0; s < 3; ++s) JiT[r][s] = (float)JiTd[r][s];
            const float om = 1.0f - chi;
            const float taf = (float)ta, tbf = (float)tb;
            // the cell in the Gauss-point buffer (rows padded to nxp cells)
            const int gl = c - (int)b.off;
            const int gc = (int)b.goff + gl + ((b.nxp == b.nx) ? 0 : (b.nxp - b.nx) * (gl / b.nx));
    #pragma unroll 2
            for (int u = 0; u < 6; ++u) {
                v4f y = {0, 0, 0, 0};
    #pragma unroll
                for (int s = 0; s < 2; ++s) y = mma3(Kb, kBfOffA2 + u * 2 + s, ch[s], cl2[s], y);
                const int q = u >> 1;
                const float xq = (u & 1) ? 0.5f : -0.5f;
                const float x0 = (q == 0) ? xq : taf;
                const float x1 = (q == 1) ? xq : ((q == 0) ? taf : tbf);
                const float x2 = (q == 2) ? xq : tbf;
                // the deviation from the cell average in FP32, added to the FP64 average
                const float dv = chi * y[0] + om * (bbar[0] * x0 + bbar[1] * x1 + bbar[2] * x2);
                const float r0 = chi * y[1] + om * bbar[0], r1 = chi * y[2] + om * bbar[1],
                            r2 = chi * y[3] + om * bbar[2];
                // face u is the + face of this cell (side 0) or the + face of the - neighbour (side 1)
                const int side = (u & 1) ? 0 : 1;
                // face record in the Gauss-point buffer: this cell's (+ face) or the minus
                // neighbour's, periodic in the block (its offset from the cell's sign of cn.dm)
                const int f = (u & 1) ? gc
                                      : gc + ((q == 0)   ? cn.dm[0]
                                              : (q == 1) ? ((cn.dm[1] < 0) ? -b.nxp : (b.ny - 1) * b.nxp)
                                                         : ((cn.dm[2] < 0) ? -b.ny * b.nxp : (b.nz - 1) * b.ny * b.nxp));
                if (valid) {
                    const long gs = b.gstride;
                    TG *dst = gp + ((long)(((q * 2 + side) * 4 + g) * 20 + v * 4)) * gs + f;
                    __builtin_nontemporal_store((TG)(q0 + (double)dv), dst);
                    __builtin_nontemporal_store((TG)(JiT[0][0] * r0 + JiT[0][1] * r1 + JiT[0][2] * r2), dst + gs);
                    __builtin_nontemporal_store((TG)(JiT[1][0] * r0 + JiT[1][1] * r1 + JiT[1][2] * r2), dst + 2 * gs);
                    __builtin_nontemporal_store((TG)(JiT[2][0] * r0 + JiT[2][1] * r1 + JiT[2][2] * r2), dst + 3 * gs);
                }
            }
        }
    }
}

hipError_t launch_recon_mfma(int prec, bool gp32, const WorkList &W, long Ntot, const double *Q, const double *G,
                             const double *L, const Metrics &M, const double *Kblk, const DevParams &P, void *gp,
                             int ngroups, const BlendIO &io, bool exp, bool stg, hipStream_t s) {
    // prec: 0 FP64, 1 FP32x3, 2 BF16x3 (Kblk holds the blocks packed for that instruction).
    // A workgroup takes whole tiles; ngroups <= 0 launches one workgroup per tile.  Learned
    // weights (P.weights = 1) and the export exist for the FP64 reconstruction only.  stg: the
    // tiles are bricks that fit kStgCells with their halo (checked by the caller), gathered
    // through LDS (FP64 and FP32x3 only).  One kernel form serves periodic blocks and blocks
    // with wall sides.
    if (W.ntiles <= 0) return hipSuccess;
    if ((P.weights == 1 || exp) && prec != 0) return hipErrorInvalidValue;
    if (exp && gp32) return hipErrorInvalidValue;
    if (stg && prec == 2) return hipErrorInvalidValue;
    const int grid = (ngroups <= 0 || ngroups > W.ntiles) ? W.ntiles : ngroups;
    const dim3 gr((unsigned)grid), bl(512);
#define CGKS_RECON(PRC, TGT, WMV, EXV)                                                                     \
    do {                                                                                                   \
        if (stg)                                                                                           \
            hipLaunchKernelGGL((k_recon_mfma<PRC, TGT, WMV, EXV, true, kStgThreads>), gr, dim3(kStgThreads), \
                               0, s, W, Ntot, Q, G, L, M, Kblk, P, (TGT *)gp, io);                         \
        else                                                                                               \
            hipLaunchKernelGGL((k_recon_mfma<PRC, TGT, WMV, EXV, false>), gr, bl, 0, s, W, Ntot, Q, G, L, M, \
                               Kblk, P, (TGT *)gp, io);                                                    \
    } while (0)
    if (prec == 0 && !gp32) {
        if (P.weights == 1) {
            if (exp) CGKS_RECON(PrecF64, double, 1, true);
            else CGKS_RECON(PrecF64, double, 1, false);
        } else {
            if (exp) CGKS_RECON(PrecF64, double, 0, true);
            else CGKS_RECON(PrecF64, double, 0, false);
        }
    } else if (prec == 0) {
        if (P.weights == 1) CGKS_RECON(PrecF64, float, 1, false);
        else CGKS_RECON(PrecF64, float, 0, false);
    } else if (prec == 1) {
        CGKS_RECON(PrecF32x3, float, 0, false);
    } else {
        hipLaunchKernelGGL((k_recon_bf16<float>), gr, bl, 0, s, W, Ntot, Q, G, L, M, Kblk, P, (float *)gp);
    }
#undef CGKS_RECON
    return hipGetLastError();
}

}  // namespace cgks
