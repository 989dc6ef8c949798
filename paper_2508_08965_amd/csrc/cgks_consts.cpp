// Constant matrices of the shared standard cell (host, FP64).
//
// The paper maps every cell to one standard cell and reconstructs there, so a single
// coefficient matrix serves all cells (Sec. 4, last paragraph).  This file builds it:
//   * the zero-mean quartic basis p_d = xi^d/d! - mean over the cell, 1 <= |d| <= 4
//     (Sec. 3.3, eq. base), in reference units (h = 1, cell [-1/2, 1/2]^3);
//   * the 72 x 34 system of eq. compact-big-ref on the unit-cube stencil: averages over the
//     6 face and 12 edge neighbours, averaged gradients of the face neighbours (weight
//     h1' = 2), averaged tangential/diagonal directional derivatives of the edge neighbours
//     (weight h2' = 1), and the 12 line differences (weight h3' = 3);
//   * its constrained least-squares solution operator R (a = R b): the face-neighbour
//     averages hold exactly, the other 66 rows in the weighted least-squares sense.
//     Solved by the null-space method with Householder QR (own implementation);
//   * point values and reference gradients of the basis at the 24 face Gauss points;
//   * Gram matrices of the smoothness indicators: first derivatives (IS^L), derivatives of
//     order 2..4 (IS^tau) and all orders (IS^H) (Sec. 3.3), by 5-point Gauss quadrature.
//
// Every integral is evaluated by Gauss-Legendre quadrature, exact for the polynomial degrees
// involved.
#include <cmath>
#include <cstring>
#include <vector>

#include "cgks_internal.h"

namespace {

using cgks::kNB;
using cgks::kNR;
using cgks::kNGP;

struct Basis {
    int d[kNB][3];
    double mean[kNB];
};

double ipow(double x, int n) {
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

double factorial(int n) {
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

// Gauss-Legendre points / weights on [-1/2, 1/2]
const double kG3x[3] = {-0.5 * 0.77459666924148337704, 0.0, 0.5 * 0.77459666924148337704};
const double kG3w[3] = {0.5 * 5.0 / 9.0, 0.5 * 8.0 / 9.0, 0.5 * 5.0 / 9.0};
const double kG5x[5] = {-0.5 * 0.90617984593866399280, -0.5 * 0.53846931010568309104, 0.0,
                        0.5 * 0.53846931010568309104, 0.5 * 0.90617984593866399280};
const double kG5w[5] = {0.5 * 0.23692688505618908751, 0.5 * 0.47862867049936646804,
                        0.5 * 0.56888888888888888889, 0.5 * 0.47862867049936646804,
                        0.5 * 0.23692688505618908751};

// d^l/dx^l of x^n / n! at x, times nothing else: x^(n-l)/(n-l)! or 0
double dmono(int n, int l, double x) {
    if (l > n) return 0.0;
    return ipow(x, n - l) / factorial(n - l);
}

// average over the unit cube centred at o of (D^l of xi^d/d!)
double cube_avg(const int d[3], const int l[3], const double o[3]) {
    double r = 1.0;
    for (int q = 0; q < 3; ++q) {
        double s = 0.0;
        for (int i = 0; i < 3; ++i) s += kG3w[i] * dmono(d[q], l[q], o[q] + kG3x[i]);
        r *= s;
    }
    return r;
}

double point_val(const int d[3], const int l[3], const double x[3]) {
    double r = 1.0;
    for (int q = 0; q < 3; ++q) r *= dmono(d[q], l[q], x[q]);
    return r;
}

void make_basis(Basis &B) {
    int n = 0;
    for (int deg = 1; deg <= 4; ++deg)
        for (int d2 = 0; d2 <= deg; ++d2)
            for (int d1 = 0; d1 <= deg - d2; ++d1) {
                B.d[n][0] = deg - d1 - d2;
                B.d[n][1] = d1;
                B.d[n][2] = d2;
                ++n;
            }
    const int l0[3] = {0, 0, 0};
    const double o0[3] = {0, 0, 0};
    for (int i = 0; i < kNB; ++i) B.mean[i] = cube_avg(B.d[i], l0, o0);
}

// Householder QR of an m x n column-major matrix A (m >= n), in place: on return A holds R in
// its upper triangle; Q (m x m, column-major) is formed explicitly.
void householder_qr(int m, int n, std::vector<double> &A, std::vector<double> &Q) {
    Q.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
    std::vector<double> v(m);
    for (int k = 0; k < n; ++k) {
        double norm = 0.0;
        for (int i = k; i < m; ++i) norm += A[(size_t)k * m + i] * A[(size_t)k * m + i];
        norm = std::sqrt(norm);
        if (norm == 0.0) continue;
        double alpha = A[(size_t)k * m + k] > 0 ? -norm : norm;
        for (int i = 0; i < m; ++i) v[i] = 0.0;
        for (int i = k; i < m; ++i) v[i] = A[(size_t)k * m + i];
        v[k] -= alpha;
        double vn = 0.0;
        for (int i = k; i < m; ++i) vn += v[i] * v[i];
        if (vn == 0.0) continue;
        for (int j = k; j < n; ++j) {  // A <- (I - 2 v v^T / v^T v) A
            double s = 0.0;
            for (int i = k; i < m; ++i) s += v[i] * A[(size_t)j * m + i];
            s = 2.0 * s / vn;
            for (int i = k; i < m; ++i) A[(size_t)j * m + i] -= s * v[i];
        }
        for (int r = 0; r < m; ++r) {  // Q <- Q (I - 2 v v^T / v^T v)
            double s = 0.0;
            for (int i = k; i < m; ++i) s += Q[(size_t)i * m + r] * v[i];
            s = 2.0 * s / vn;
            for (int i = k; i < m; ++i) Q[(size_t)i * m + r] -= s * v[i];
        }
    }
}

}  // namespace

namespace cgks {

void build_constants(HostConsts &K) {
    Basis B;
    make_basis(B);
    const double g = 0.5 / std::sqrt(3.0);

    // ---- rows of the standard-cell system, weighted ------------------------------------
    double A[kNR][kNB];
    double w[kNR];
    for (int r = 0; r < kNR; ++r) w[r] = 1.0;
    const int zero[3] = {0, 0, 0};
    for (int i = 0; i < kNB; ++i) {
        for (int m = 0; m < 6; ++m) {
            double o[3] = {0, 0, 0};
            o[m / 2] = (m & 1) ? 1.0 : -1.0;
            A[m][i] = cube_avg(B.d[i], zero, o) - B.mean[i];
            for (int j = 0; j < 3; ++j) {
                int l[3] = {0, 0, 0};
                l[j] = 1;
                A[kRowFaceGrad + 3 * m + j][i] = cube_avg(B.d[i], l, o);
                w[kRowFaceGrad + 3 * m + j] = 2.0;
            }
        }
        for (int n = 0; n < 12; ++n) {
            EdgeDef e = edge_def(n);
            A[kRowEdgeAvg + n][i] = cube_avg(B.d[i], zero, e.off) - B.mean[i];
            double s1 = 0, s2 = 0;
            for (int j = 0; j < 3; ++j) {
                int l[3] = {0, 0, 0};
                l[j] = 1;
                double v = cube_avg(B.d[i], l, e.off);
                s1 += e.t1[j] * v;
                s2 += e.t2[j] * v;
            }
            A[kRowEdgeDir + 2 * n][i] = s1;
            A[kRowEdgeDir + 2 * n + 1][i] = s2;
        }
        for (int s = 0; s < 12; ++s) {
            int q = s / 4, k = s % 4;
            double xm[3], xp[3];
            int a = (q == 0) ? 1 : 0, b = (q == 2) ? 1 : 2;
            xm[a] = xp[a] = (2 * (k & 1) - 1) * g;
            xm[b] = xp[b] = (2 * (k >> 1) - 1) * g;
            xm[q] = -0.5;
            xp[q] = 0.5;
            A[kRowLine + s][i] = point_val(B.d[i], zero, xp) - point_val(B.d[i], zero, xm);
            w[kRowLine + s] = 3.0;
        }
    }

    // ---- null-space method: C a = bC (6 rows), min |W (AL a - bL)| ---------------------
    const int nc = 6, nl = kNR - 6;
    std::vector<double> Ct((size_t)kNB * nc), Qc;
    for (int r = 0; r < nc; ++r)
        for (int i = 0; i < kNB; ++i) Ct[(size_t)r * kNB + i] = A[r][i];  // column r of C^T
    householder_qr(kNB, nc, Ct, Qc);
    // R1 (6x6 upper) = Ct upper block; Y = Qc[:, 0:6], Z = Qc[:, 6:34]
    auto Y = [&](int i, int j) { return Qc[(size_t)j * kNB + i]; };
    auto Z = [&](int i, int j) { return Qc[(size_t)(nc + j) * kNB + i]; };
    const int nz = kNB - nc;
    // M = W AL Z (nl x nz), column-major
    std::vector<double> M((size_t)nl * nz), Qm;
    for (int j = 0; j < nz; ++j)
        for (int r = 0; r < nl; ++r) {
            double s = 0.0;
            for (int i = 0; i < kNB; ++i) s += A[nc + r][i] * Z(i, j);
            M[(size_t)j * nl + r] = w[nc + r] * s;
        }
    householder_qr(nl, nz, M, Qm);
    for (int col = 0; col < kNR; ++col) {
        double bc[6] = {0, 0, 0, 0, 0, 0};
        std::vector<double> bl(nl, 0.0);
        if (col < nc) bc[col] = 1.0;
        else bl[col - nc] = 1.0;
        // u = R1^{-T} bc  (R1^T lower triangular: forward substitution)
        double u[6];
        for (int i = 0; i < nc; ++i) {
            double s = bc[i];
            for (int j = 0; j < i; ++j) s -= Ct[(size_t)i * kNB + j] * u[j];
            u[i] = s / Ct[(size_t)i * kNB + i];
        }
        double ap[kNB];
        for (int i = 0; i < kNB; ++i) {
            double s = 0.0;
            for (int j = 0; j < nc; ++j) s += Y(i, j) * u[j];
            ap[i] = s;
        }
        // rhs = Qm^T W (bl - AL ap), first nz entries
        std::vector<double> rhs(nl);
        for (int r = 0; r < nl; ++r) {
            double s = 0.0;
            for (int i = 0; i < kNB; ++i) s += A[nc + r][i] * ap[i];
            rhs[r] = w[nc + r] * (bl[r] - s);
        }
        double y[kNB];
        std::vector<double> t(nz);
        for (int j = 0; j < nz; ++j) {
            double s = 0.0;
            for (int r = 0; r < nl; ++r) s += Qm[(size_t)j * nl + r] * rhs[r];
            t[j] = s;
        }
        for (int j = nz - 1; j >= 0; --j) {  // back substitution with Rm
            double s = t[j];
            for (int k = j + 1; k < nz; ++k) s -= M[(size_t)k * nl + j] * y[k];
            y[j] = s / M[(size_t)j * nl + j];
        }
        for (int i = 0; i < kNB; ++i) {
            double s = ap[i];
            for (int j = 0; j < nz; ++j) s += Z(i, j) * y[j];
            K.R[i][col] = s;
        }
    }

    // ---- basis at the 24 face Gauss points: value and reference gradient --------------
    for (int m = 0; m < 6; ++m)
        for (int k = 0; k < 4; ++k) {
            int gp = 4 * m + k, q = m / 2;
            int a = (q == 0) ? 1 : 0, b = (q == 2) ? 1 : 2;
            double x[3];
            x[q] = (m & 1) ? 0.5 : -0.5;
            x[a] = (2 * (k & 1) - 1) * g;
            x[b] = (2 * (k >> 1) - 1) * g;
            for (int j = 0; j < 3; ++j) K.xg[gp][j] = x[j];
            for (int i = 0; i < kNB; ++i) {
                K.E[gp][0][i] = point_val(B.d[i], zero, x) - B.mean[i];
                for (int j = 0; j < 3; ++j) {
                    int l[3] = {0, 0, 0};
                    l[j] = 1;
                    K.E[gp][1 + j][i] = point_val(B.d[i], l, x);
                }
            }
        }

    // ---- basis at the 3^3 Gauss points of the cell (volume integrals of the diagnostics) --
    for (int gv = 0; gv < 27; ++gv) {
        const int ix[3] = {gv % 3, (gv / 3) % 3, gv / 9};
        double x[3];
        K.wv[gv] = 1.0;
        for (int j = 0; j < 3; ++j) {
            x[j] = kG3x[ix[j]];
            K.xv[gv][j] = x[j];
            K.wv[gv] *= kG3w[ix[j]];
        }
        for (int i = 0; i < kNB; ++i) {
            K.V[gv][0][i] = point_val(B.d[i], zero, x) - B.mean[i];
            for (int j = 0; j < 3; ++j) {
                int l[3] = {0, 0, 0};
                l[j] = 1;
                K.V[gv][1 + j][i] = point_val(B.d[i], l, x);
            }
        }
    }

    // ---- Gram matrices of the smoothness indicators -------------------------------------
    std::memset(K.GL, 0, sizeof K.GL);
    std::memset(K.GT, 0, sizeof K.GT);
    for (int l0 = 0; l0 <= 4; ++l0)
        for (int l1 = 0; l1 <= 4 - l0; ++l1)
            for (int l2 = 0; l2 <= 4 - l0 - l1; ++l2) {
                int ord = l0 + l1 + l2;
                if (ord == 0) continue;
                int l[3] = {l0, l1, l2};
                for (int i = 0; i < kNB; ++i)
                    for (int j = 0; j < kNB; ++j) {
                        double s = 0.0;
                        for (int a = 0; a < 5; ++a)
                            for (int b = 0; b < 5; ++b)
                                for (int c = 0; c < 5; ++c) {
                                    double x[3] = {kG5x[a], kG5x[b], kG5x[c]};
                                    s += kG5w[a] * kG5w[b] * kG5w[c] * point_val(B.d[i], l, x) *
                                         point_val(B.d[j], l, x);
                                }
                        if (ord == 1) K.GL[i][j] += s;
                        else K.GT[i][j] += s;
                    }
            }
    for (int i = 0; i < kNB; ++i)
        for (int j = 0; j < kNB; ++j) K.GH[i][j] = K.GL[i][j] + K.GT[i][j];
}

}  // namespace cgks

namespace cgks {

namespace {

// lower-triangular Cholesky factor of an n x n SPD matrix (row-major), in place into Lo
bool cholesky(int n, const double *A, double *Lo) {
    for (int i = 0; i < n * n; ++i) Lo[i] = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= Lo[j * n + k] * Lo[j * n + k];
        if (!(s > 0.0)) return false;
        const double d = std::sqrt(s);
        Lo[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= Lo[i * n + k] * Lo[j * n + k];
            Lo[i * n + j] = t / d;
        }
    }
    return true;
}

// stencil item of k index 4s+g in the matrix-core order of the reconstruction kernel
int mfma_item(int k) {
    const int s = k / 4, g = k % 4;
    if (s < 6) return (g == 0) ? s : kRowFaceGrad + 3 * s + (g - 1);
    if (s < 9) return kRowEdgeAvg + 4 * (s - 6) + g;
    if (s < 15) {
        const int p = (s - 9) / 2, d = (s - 9) % 2;
        return kRowEdgeDir + 2 * (4 * p + g) + d;
    }
    return kRowLine + 4 * (s - 15) + g;
}

// Output layout of the 16x16x4 instructions: register v of lane l holds row
//   f32: 4 (l/16) + v          f64: 4 v + l/16          (column l % 16 in both).
// Row of the quartic coefficient vector held in register v of GEMM1 tile t by lane group g,
// i.e. the contraction index 4s'+g of the follow-up products, s' = 4t+v.
int mfma_arow(int sp, int g, bool f64) {
    const int t = sp / 4, v = sp % 4;
    return 16 * t + (f64 ? 4 * v + g : 4 * g + v);
}

}  // namespace

namespace {

// FP64 layout: the coefficients ordered by parity class (odd or even in x, y, z), the
// classes in the order of kParityClass; within a class the basis order.  The first members of
// OEE, EOE and EEO are x, y and z (the degree-1 monomials).
constexpr int kParityClass[8] = {1, 2, 4, 3, 5, 6, 0, 7};  // bit q set: odd in axis q
bool parity_order(int perm[kNB]) {
    Basis B;
    make_basis(B);
    int n = 0;
    for (int c : kParityClass)
        for (int i = 0; i < kNB; ++i) {
            const int cls = (B.d[i][0] & 1) | ((B.d[i][1] & 1) << 1) | ((B.d[i][2] & 1) << 2);
            if (cls == c) perm[n++] = i;
        }
    // the k-step lists the FP64 kernel compiles in (groups of 4 coefficients, one class per
    // group but for the last, which holds the ninth even-even-even coefficient and the
    // odd-odd-odd one)
    static const int kClassOfStep[8] = {1, 2, 4, 3, 5, 6, 0, 0};
    for (int k = 0; k < 32; ++k) {
        const int *d = B.d[perm[k]];
        if (((d[0] & 1) | ((d[1] & 1) << 1) | ((d[2] & 1) << 2)) != kClassOfStep[k / 4]) return false;
    }
    const int *d32 = B.d[perm[32]], *d33 = B.d[perm[33]];
    return n == kNB && (d32[0] | d32[1] | d32[2]) % 2 == 0 && (d33[0] & d33[1] & d33[2] & 1) &&
           perm[0] == 0 && perm[4] == 1 && perm[8] == 2;
}

// Cholesky factor of the Gram matrix G restricted to the index list idx (in that order), with
// the entries between different parity classes, zero on the centred cell up to the rounding
// of the quadrature sums, set to zero
bool cholesky_sub(const Basis &B, const double G[kNB][kNB], const std::vector<int> &idx, std::vector<double> &Lo) {
    const int n = (int)idx.size();
    std::vector<double> A((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const int *di = B.d[idx[i]], *dj = B.d[idx[j]];
            const bool same = (((di[0] ^ dj[0]) | (di[1] ^ dj[1]) | (di[2] ^ dj[2])) & 1) == 0;
            if (!same && std::fabs(G[idx[i]][idx[j]]) > 1e-13) return false;
            A[(size_t)i * n + j] = same ? G[idx[i]][idx[j]] : 0.0;
        }
    Lo.assign((size_t)n * n, 0.0);
    return cholesky(n, A.data(), Lo.data());
}

// FP64 packing in the parity order (see the kernel): R rows permuted; L_L^T and L_T^T of the
// permuted Gram matrices (block diagonal: products of different classes integrate to zero on
// the centred cell); per face pair q the even and odd parts of the + face's E rows, from which
// both faces follow (the - face's rows are the + face's times (-1)^(exponent of axis q), the
// normal derivative with the opposite sign), checked here against the - face's own rows.
bool pack_mfma_parity(const HostConsts &K, double *blk) {
    int perm[kNB];
    if (!parity_order(perm)) return false;
    Basis B;
    make_basis(B);
    std::vector<int> all(kNB), nonlin;
    for (int n = 0; n < kNB; ++n) {
        all[n] = perm[n];
        if (n != 0 && n != 4 && n != 8) nonlin.push_back(perm[n]);
    }
    std::vector<double> ll, lt;
    if (!cholesky_sub(B, K.GL, all, ll) || !cholesky_sub(B, K.GT, nonlin, lt)) return false;
    // coefficient position (new index) of row r of L_T^T: the non-linear coefficients in order
    int tpos[31];
    for (int r = 0, n = 0; n < kNB; ++n)
        if (n != 0 && n != 4 && n != 8) tpos[r++] = n;
    for (int i = 0; i < kMfmaBlocks * 64; ++i) blk[i] = 0.0;
    for (int l = 0; l < 64; ++l) {
        const int row = l % 16, g = l / 16;
        for (int t = 0; t < 3; ++t)
            for (int s = 0; s < 18; ++s) {
                const int i = 16 * t + row;
                blk[(kMfmaOffA1 + t * 18 + s) * 64 + l] = (i < kNB) ? K.R[perm[i]][mfma_item(4 * s + g)] : 0.0;
            }
        for (int s = 0; s < 9; ++s) {
            const int ar = 4 * s + g;  // coefficient (new index) of k-step s, lane group g
            for (int u = 0; u < 3; ++u) {
                const int i = 16 * u + row;  // row of L_L^T
                blk[(kMfmaOffAL + u * 10 + s) * 64 + l] = (i < kNB && ar < kNB) ? ll[(size_t)ar * kNB + i] : 0.0;
            }
            for (int u = 0; u < 2; ++u) {
                const int r = 16 * u + row;  // row of L_T^T (non-linear coefficient r)
                double v = 0.0;
                if (r < 31 && ar < kNB)
                    for (int c = 0; c < 31; ++c)
                        if (tpos[c] == ar) v = lt[(size_t)c * 31 + r];
                blk[(kMfmaOffAT + u * 10 + s) * 64 + l] = v;
            }
        }
        // E: pair q, even steps (6) then odd steps (4) of kParityEven / kParityOdd
        static const int kEven[3][6] = {{1, 2, 5, 6, 7, 8}, {0, 2, 4, 6, 7, 8}, {0, 1, 3, 6, 7, 8}};
        static const int kOdd[3][4] = {{0, 3, 4, 8}, {1, 3, 5, 8}, {2, 4, 5, 8}};
        const int gpl = row % 4, comp = row / 4;
        for (int q = 0; q < 3; ++q)
            for (int j = 0; j < 10; ++j) {
                const int s = (j < 6) ? kEven[q][j] : kOdd[q][j - 6];
                const int ar = 4 * s + g;
                double v = 0.0;
                if (ar < kNB) {
                    const bool odd = (B.d[perm[ar]][q] & 1) != 0;
                    if (odd == (j >= 6)) v = K.E[4 * (2 * q + 1) + gpl][comp][perm[ar]];
                }
                blk[(kMfmaOffA2 + q * 10 + j) * 64 + l] = v;
            }
    }
    // the smoothness-form tiles read only k-steps [kISFrom, kISTo): every other block is zero
    static const int kISFrom[5] = {0, 4, 8, 0, 4}, kISTo[5] = {4, 9, 9, 5, 9};
    for (int u = 0; u < 5; ++u)
        for (int st = 0; st < 10; ++st)
            if (st < kISFrom[u] || st >= kISTo[u]) {
                const int base = (u < 3) ? kMfmaOffAL + u * 10 : kMfmaOffAT + (u - 3) * 10;
                for (int l = 0; l < 64; ++l)
                    if (blk[(base + st) * 64 + l] != 0.0) return false;
            }
    // the - face of each pair from the + face's rows
    for (int q = 0; q < 3; ++q)
        for (int gp = 0; gp < 4; ++gp)
            for (int comp = 0; comp < 4; ++comp)
                for (int i = 0; i < kNB; ++i) {
                    const double sgn = ((B.d[i][q] & 1) ? -1.0 : 1.0) * ((comp == 1 + q) ? -1.0 : 1.0);
                    const double want = K.E[4 * (2 * q) + gp][comp][i], have = sgn * K.E[4 * (2 * q + 1) + gp][comp][i];
                    if (std::fabs(want - have) > 1e-13 * (1.0 + std::fabs(want))) return false;
                }
    return true;
}

}  // namespace

bool pack_mfma(const HostConsts &K, double *blk, bool f64) {
    if (f64) return pack_mfma_parity(K, blk);
    // Cholesky factors of the Gram matrices: IS^L = |L_L^T a|^2 over all 34 coefficients,
    // IS^tau = |L_T^T a_s|^2 over the 31 coefficients of degree >= 2 (indices 3..33)
    std::vector<double> gl(kNB * kNB), ll(kNB * kNB), gt(31 * 31), lt(31 * 31);
    for (int i = 0; i < kNB; ++i)
        for (int j = 0; j < kNB; ++j) gl[i * kNB + j] = K.GL[i][j];
    for (int i = 0; i < 31; ++i)
        for (int j = 0; j < 31; ++j) gt[i * 31 + j] = K.GT[3 + i][3 + j];
    if (!cholesky(kNB, gl.data(), ll.data()) || !cholesky(31, gt.data(), lt.data())) return false;
    for (int i = 0; i < kMfmaBlocks * 64; ++i) blk[i] = 0.0;
    for (int l = 0; l < 64; ++l) {
        const int row = l % 16, g = l / 16;
        for (int t = 0; t < 3; ++t)
            for (int s = 0; s < 18; ++s) {
                const int i = 16 * t + row;
                blk[(kMfmaOffA1 + t * 18 + s) * 64 + l] = (i < kNB) ? K.R[i][mfma_item(4 * s + g)] : 0.0;
            }
        for (int s = 0; s < 10; ++s) {
            const int ar = mfma_arow(s, g, f64);
            for (int u = 0; u < 3; ++u) {
                const int i = 16 * u + row;  // row of L_L^T
                blk[(kMfmaOffAL + u * 10 + s) * 64 + l] = (i < kNB && ar < kNB) ? ll[ar * kNB + i] : 0.0;
            }
            for (int u = 0; u < 2; ++u) {
                const int i = 16 * u + row;  // row of L_T^T (sub-indices)
                blk[(kMfmaOffAT + u * 10 + s) * 64 + l] = (i < 31 && ar >= 3 && ar < kNB) ? lt[(ar - 3) * 31 + i] : 0.0;
            }
            for (int u = 0; u < 6; ++u) {
                // output rows of a tile: lane group = Gauss point, register = component
                const int gpl = f64 ? row % 4 : row / 4, comp = f64 ? row / 4 : row % 4;
                blk[(kMfmaOffA2 + u * 10 + s) * 64 + l] = (ar < kNB) ? K.E[4 * u + gpl][comp][ar] : 0.0;
            }
        }
    }
    return true;
}

}  // namespace cgks

namespace cgks {

bool pack_mfma_bf16(const HostConsts &K, double *blk) {
    // Cholesky factors as in pack_mfma
    std::vector<double> gl(kNB * kNB), ll(kNB * kNB), gt(31 * 31), lt(31 * 31);
    for (int i = 0; i < kNB; ++i)
        for (int j = 0; j < kNB; ++j) gl[i * kNB + j] = K.GL[i][j];
    for (int i = 0; i < 31; ++i)
        for (int j = 0; j < 31; ++j) gt[i * 31 + j] = K.GT[3 + i][3 + j];
    if (!cholesky(kNB, gl.data(), ll.data()) || !cholesky(31, gt.data(), lt.data())) return false;
    for (int i = 0; i < kBfBlocks * 512; ++i) blk[i] = 0.0;
    // item slot sigma = 8 s + j of lane group g is the uniform slot of the 16x16x4 kernels,
    // i.e. stencil item mfma_item(4 sigma + g); slots 18..23 are padding
    // coefficient slot sigma' = 8 s' + j of lane group g holds a-row 16 t + 4 g + v, (t, v) =
    // (sigma' / 4, sigma' % 4), for sigma' < 12
    auto arow = [](int sp, int j, int g) -> int {
        const int sig = 8 * sp + j;
        if (sig >= 12) return -1;
        return 16 * (sig / 4) + 4 * g + (sig % 4);
    };
    for (int l = 0; l < 64; ++l) {
        const int row = l % 16, g = l / 16;
        for (int j = 0; j < 8; ++j) {
            for (int t = 0; t < 3; ++t)
                for (int s = 0; s < 3; ++s) {
                    const int sig = 8 * s + j, i = 16 * t + row;
                    const double v = (sig < 18 && i < kNB) ? K.R[i][mfma_item(4 * sig + g)] : 0.0;
                    blk[((kBfOffA1 + t * 3 + s) * 64 + l) * 8 + j] = v;
                }
            for (int s = 0; s < 2; ++s) {
                const int ar = arow(s, j, g);
                for (int u = 0; u < 3; ++u) {
                    const int i = 16 * u + row;
                    blk[((kBfOffAL + u * 2 + s) * 64 + l) * 8 + j] = (ar >= 0 && ar < kNB && i < kNB) ? ll[ar * kNB + i] : 0.0;
                }
                for (int u = 0; u < 2; ++u) {
                    const int i = 16 * u + row;
                    blk[((kBfOffAT + u * 2 + s) * 64 + l) * 8 + j] =
                        (ar >= 3 && ar < kNB && i < 31) ? lt[(ar - 3) * 31 + i] : 0.0;
                }
                for (int u = 0; u < 6; ++u) {
                    const int gpl = row / 4, comp = row % 4;  // FP32-layout output rows
                    blk[((kBfOffA2 + u * 2 + s) * 64 + l) * 8 + j] = (ar >= 0 && ar < kNB) ? K.E[4 * u + gpl][comp][ar] : 0.0;
                }
            }
        }
    }
    return true;
}

}  // namespace cgks
