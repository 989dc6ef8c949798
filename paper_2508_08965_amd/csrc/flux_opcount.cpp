// Source-level operation count of the gas-kinetic flux (gks_flux_pair) per Gauss point.
//
// The flux is generic in its arithmetic type; instantiating it on the host with a counting
// type gives the number of additions, multiplications, fused multiply-adds, divisions and
// transcendental calls (sqrt, exp, erfc, pow) of one lane.  Both lanes of a pair execute the
// same instruction stream (the code has no lane-dependent branches; the pair exchange is a
// value swap), so the hardware issues twice the count of one lane per Gauss point.  Part of
// that stream is the same on both lanes (the face frame, the pair sums, the equilibrium
// state and its slopes, the time-derivative coefficient, the collision time and the time
// integrals) or is used from one lane only (the heat-flux correction, the rotation of the
// flux back to the global frame); the template marks those sections, and the method's work
// per Gauss point counts them once: 2 x (per-side work) + 1 x (shared work).
// Prints one line:
//   <issued flops per Gauss point, stage 1> <adds> <muls> <fmas> <divs> <transcendentals>
//   <status> <issued flops, stage 2> <method flops, stage 1> <method flops, stage 2>
// (adds ... transcendentals per lane, stage 1) with flops = adds + muls + 2 fmas + divs +
// transcendentals.  Stage 2 computes only the time derivatives.
// Usage: flux_opcount [viscous] [prandtl_fix] [sutherland] [tau_zero]   (0/1 each)
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "cgks_device.h"

namespace {

struct Tally {
    long add = 0, mul = 0, fma = 0, div = 0, trans = 0;
    long flops() const { return add + mul + 2 * fma + div + trans; }
};
Tally own, shared;   // per-side work / work both lanes repeat
Tally *cur = &own;

struct Cnt {
    double v;
    Cnt() : v(0.0) {}
    Cnt(double x) : v(x) {}
};
inline Cnt operator+(Cnt a, Cnt b) { ++cur->add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++cur->add; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++cur->mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++cur->div; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt &operator+=(Cnt &a, Cnt b) { ++cur->add; a.v += b.v; return a; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }

struct HostCount {
    static Cnt swap(Cnt v) { return v; }
    static int swapi(int v) { return v; }
    static Cnt sqrt(Cnt x) { ++cur->trans; return Cnt(std::sqrt(x.v)); }
    static Cnt exp(Cnt x) { ++cur->trans; return Cnt(std::exp(x.v)); }
    static Cnt erfc(Cnt x) { ++cur->trans; return Cnt(std::erfc(x.v)); }
    static Cnt pow(Cnt a, Cnt b) { ++cur->trans; return Cnt(std::pow(a.v, b.v)); }
    static Cnt fabs(Cnt x) { return Cnt(std::fabs(x.v)); }
    static Cnt fma(Cnt a, Cnt b, Cnt c) { ++cur->fma; return Cnt(a.v * b.v + c.v); }
    static bool finite(Cnt x) { return std::isfinite(x.v); }
    static void pair_shared(bool on) { cur = on ? &shared : &own; }
};

Tally sum(const Tally &a, const Tally &b) {
    Tally t;
    t.add = a.add + b.add; t.mul = a.mul + b.mul; t.fma = a.fma + b.fma; t.div = a.div + b.div;
    t.trans = a.trans + b.trans;
    return t;
}

}  // namespace

int main(int argc, char **argv) {
    cgks::DevParams P{};
    P.gamma = 1.4;
    P.K = 2.0;
    P.tau_eps = 0.05;
    P.tau_C = 5.0;
    P.mu0 = 1.0 / 1600.0;
    P.T_ref = 71.4285714;
    P.S_suth = P.T_ref * 110.4 / 288.15;
    P.Pr = 0.72;
    P.inv_K3 = 1.0 / (P.K + 3.0);
    P.inv_Tref = 1.0 / P.T_ref;
    P.viscous = argc > 1 ? std::atoi(argv[1]) : 1;
    P.prandtl_fix = argc > 2 ? std::atoi(argv[2]) : 1;
    P.visc_law = argc > 3 ? std::atoi(argv[3]) : 1;
    P.tau_zero = argc > 4 ? std::atoi(argv[4]) : 0;
    // a physical left state with non-zero gradients and a tilted normal
    Cnt q[5] = {1.01, 0.31, -0.22, 0.05, 180.0};
    Cnt g[5][3];
    for (int v = 0; v < 5; ++v)
        for (int j = 0; j < 3; ++j) g[v][j] = Cnt(0.01 * (1 + v) * (j - 1));
    const double nn = std::sqrt(1.0 + 0.04 + 0.01);
    Cnt n[3] = {1.0 / nn, 0.2 / nn, 0.1 / nn};
    Cnt Fo[5], Fto[5], Qs[5], dQs[5];
    // full flux (first stage), then the time derivatives only (second stage)
    const int err = cgks::gks_flux_pair<HostCount, Cnt, true>(P, 0, q, g, n, Cnt(4e-4), Fo, Fto, Qs, dQs);
    const Tally lane1 = sum(own, shared);
    const long method1 = 2 * own.flops() + shared.flops();
    own = Tally{};
    shared = Tally{};
    const int err2 = cgks::gks_flux_pair<HostCount, Cnt, false>(P, 0, q, g, n, Cnt(4e-4), Fo, Fto, Qs, dQs);
    const long lane2 = sum(own, shared).flops();
    const long method2 = 2 * own.flops() + shared.flops();
    std::printf("%ld %ld %ld %ld %ld %ld %d %ld %ld %ld\n", 2 * lane1.flops(), lane1.add, lane1.mul, lane1.fma,
                lane1.div, lane1.trans, err, 2 * lane2, method1, method2);
    return err | err2;
}
