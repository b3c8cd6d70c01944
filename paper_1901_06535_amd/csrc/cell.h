// cell.h -- the per-cell forward-Euler update of the Oregonator (Sec. 2,
// Eq. (1)), shared by every kernel of one precision so that all launch
// shapes (one step per launch, T steps per launch, any tile height) produce
// bit-identical fields.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rdc {

// Scheme constants in the working precision, formed once in double on the
// host: c1 = dt/eps scales the reaction bracket, c2 = dt*D_u/dx^2 the
// five-node sum.  The FP32 update also uses the regrouped constants
// k0 = 1 + c1 - 4 c2, c1f = c1 f and omdt = 1 - dt.
template <typename Real>
struct Consts {
    Real c1, c2, f, q, dt;
    Real k0, c1f, omdt;
};

// FP32 update.  The forward-Euler step of Eq. (1),
//   u' = u + c1 [u - u^2 - (f v + phi)(u - q)/(u + q)] + c2 (s - 4u),
//   v' = v + dt (u - v),
// regrouped to take few instructions per cell:
//   u' = u (k0 - c1 u) + c2 s - G (u - q)/(u + q),   G = c1 f v + c1 phi,
//   v' = dt u + (1 - dt) v.
// c1 phi arrives precomputed (`c1phi`, one FP32 multiply of the cell's phi),
// the quotient is the hardware reciprocal of (u + q) (about 1 ulp) times the
// numerator.  Contraction is pinned (fmaf where written, nowhere else), so
// every kernel that calls this gets bit-identical results.
__device__ __forceinline__ void cell_update(float uC, float uW, float uE, float uN, float uS,
                                            float vC, float c1phi, const Consts<float>& k,
                                            float& u_next, float& v_next) {
#pragma clang fp contract(off)
    const float s = (uW + uE) + (uN + uS);                   // west+east first: D4-symmetric
    const float t1 = __builtin_fmaf(-k.c1, uC, k.k0);        // k0 - c1 u
    const float A = __builtin_fmaf(t1, uC, k.c2 * s);        // u (k0 - c1 u) + c2 s
    const float G = __builtin_fmaf(k.c1f, vC, c1phi);        // c1 (f v + phi)
    const float h = G * __builtin_amdgcn_rcpf(uC + k.q);     // G / (u + q)
    u_next = __builtin_fmaf(-h, uC, __builtin_fmaf(h, k.q, A));  // A - h (u - q)
    v_next = __builtin_fmaf(k.dt, uC, k.omdt * vC);
}

// c1 * phi as the FP32 update takes it (one rounding, the same in every kernel).
__device__ __forceinline__ float scaled_phi(float phi, const Consts<float>& k) {
#pragma clang fp contract(off)
    return k.c1 * phi;
}

// FP64 update: one fixed order of operations with no contraction and IEEE
// division, so that it reproduces a plain C evaluation of the same
// expressions bit for bit:
//   s = (uW + uE) + (uN + uS);  lap = s - 4 uC;  a = uC - uC*uC;
//   g = f vC + phiC;  r = (uC - q)/(uC + q);  Ru = a - g r;
//   u' = (uC + c1 Ru) + c2 lap;  v' = vC + dt (uC - vC).
__device__ __forceinline__ void cell_update(double uC, double uW, double uE, double uN,
                                            double uS, double vC, double phiC,
                                            const Consts<double>& k, double& u_next,
                                            double& v_next) {
#pragma clang fp contract(off)
    const double s = (uW + uE) + (uN + uS);
    const double lap = s - 4.0 * uC;
    const double a = uC - uC * uC;
    const double g = k.f * vC + phiC;
    const double r = (uC - k.q) / (uC + k.q);
    const double Ru = a - g * r;
    u_next = (uC + k.c1 * Ru) + k.c2 * lap;
    v_next = vC + k.dt * (uC - vC);
}

// The FP64 update takes phi itself.
__device__ __forceinline__ double scaled_phi(double phi, const Consts<double>&) { return phi; }

// Index of the cell whose value a position i (possibly outside [0, n))
// takes under the no-flux edge: the even extension mirrored about each cell
// face, repeated with period 2n.  Within one cell of the edge this is the
// "neighbour = edge cell" ghost; further out it is the value the ghost region
// would evolve to, which is what lets a tile's halo run several steps with no
// per-step edge handling.
__device__ __forceinline__ int reflect_index(int i, int n) {
    if (i >= 0 && i < n) return i;
    const int m = 2 * n;
    i %= m;
    if (i < 0) i += m;
    return i < n ? i : m - 1 - i;
}

}  // namespace rdc
