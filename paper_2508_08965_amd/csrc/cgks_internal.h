// Internal definitions shared by the host set-up and the HIP kernels of the library.
#pragma once

#include <cmath>

namespace cgks {

constexpr int kNV = 5;    // conserved variables
constexpr int kNB = 34;   // basis of the quartic, 1 <= |d| <= 4
constexpr int kNR = 72;   // stencil data per variable (rows of the standard-cell system)
constexpr int kNGP = 24;  // face Gauss points of one cell

// Row blocks of the standard-cell system (order of eq. compact-big-5 / compact-big-ref):
// face averages (exact) | edge averages | face gradients (3 per face) | edge directional
// derivatives (tau1, tau2 per edge) | line differences.
constexpr int kRowEdgeAvg = 6;
constexpr int kRowFaceGrad = 18;
constexpr int kRowEdgeDir = 36;
constexpr int kRowLine = 60;

struct EdgeDef {
    double off[3];  // offset of the edge neighbour
    double t1[3];   // unit vector along the shared edge
    double t2[3];   // unit vector from the target centroid to the neighbour centroid
};

// Edge n = 4p + (sa > 0) + 2 (sb > 0), axis pairs p: (0,1), (0,2), (1,2).
inline EdgeDef edge_def(int n) {
    static const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2}, pc[3] = {2, 1, 0};
    EdgeDef e;
    int p = n / 4;
    for (int q = 0; q < 3; ++q) e.off[q] = e.t1[q] = e.t2[q] = 0.0;
    e.off[pa[p]] = (n & 1) ? 1.0 : -1.0;
    e.off[pb[p]] = (n & 2) ? 1.0 : -1.0;
    e.t1[pc[p]] = 1.0;
    const double r = 1.0 / std::sqrt(2.0);
    for (int q = 0; q < 3; ++q) e.t2[q] = e.off[q] * r;
    return e;
}

// Constant matrices of the standard cell (host copy; uploaded once per context).
struct HostConsts {
    double R[kNB][kNR];         // a = R b
    double E[kNGP][4][kNB];     // per Gauss point: value row, then d/dxi, d/deta, d/dzeta rows
    double GH[kNB][kNB];        // Gram matrix of all derivatives 1..4  (IS^H)
    double GL[kNB][kNB];        // first derivatives                    (IS^L)
    double GT[kNB][kNB];        // derivatives 2..4                     (IS^tau)
    double xg[kNGP][3];         // reference Gauss points (centred standard cell)
    double V[27][4][kNB];       // basis value and reference gradient at the 3^3 volume Gauss points
    double xv[27][3];           // those points (centred standard cell, x fastest)
    double wv[27];              // their weights (product of 5/18, 8/18, 5/18; sum 1)
};

void build_constants(HostConsts &K);

// Constant blocks of the matrix-core reconstruction (16x16x4 instructions), 64 values per
// block in the per-lane order the instruction reads: R (3 tiles x 18 k-steps), L_L^T (3 x 10),
// L_T^T (2 x 10), E (6 x 10).  f64 selects the output layout of the FP64 instruction
// (register v of lane l holds row 4v + l/16), otherwise that of the FP32 one (row 4(l/16) + v).
constexpr int kMfmaOffA1 = 0, kMfmaOffAL = 54, kMfmaOffAT = 84, kMfmaOffA2 = 104, kMfmaBlocks = 164;
bool pack_mfma(const HostConsts &K, double *blocks, bool f64);

// Constant blocks of the BF16x3 reconstruction (16x16x32 BF16 instruction): 8 values per lane
// and block: R (3 tiles x 3 k-steps), L_L^T (3 x 2), L_T^T (2 x 2), E (6 x 2); split into
// BF16 hi/lo pairs on the device.
constexpr int kBfOffA1 = 0, kBfOffAL = 9, kBfOffAT = 15, kBfOffA2 = 19, kBfBlocks = 31;
bool pack_mfma_bf16(const HostConsts &K, double *blocks);

// Scheme parameters in the form the kernels read them.
struct DevParams {
    double gamma, K;             // ratio of specific heats, internal degrees of freedom
    double cfl, tau_eps, tau_C;
    double mu0, T_ref, S_suth, Pr;
    double geno_C, geno_eps, geno_r, inv_tanhC;
    double jump_thresh;          // pressure-jump indicator of the learned-weight fallback
    int viscous, visc_law, tau_zero, linear, prandtl_fix;
    int weights;                 // 0 GENO weights, 1 learned weights with GENO fallback
    double far[5];               // far-field state (conserved variables) of far-field sides
    double inv_K3, inv_Tref;     // 1 / (K + 3), 1 / T_ref
    int positivity;              // 1: interface-state limiter (an addition to the paper)
    double pos_eps;              // its floor, a fraction of the cell average's density, pressure
};

}  // namespace cgks
