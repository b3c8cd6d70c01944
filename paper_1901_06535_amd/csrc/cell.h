// cell.h -- the per-cell forward-Euler update of the Oregonator (Sec. 2,
// Eq. (1)), shared by every kernel of one precision so that all launch
// shapes (one step per launch, T steps per launch, any tile height) produce
// bit-identical fields.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rdc {

// Scheme constants in the working precision.  c1 = dt/eps scales the
// reaction bracket, c2 = dt*D_u/dx^2 scales the five-node sum; both are
// formed once in double on the host.
template <typename Real>
struct Consts {
    Real c1, c2, f, q, dt;
};

// FP32 update.  Contraction is pinned (fmaf where written, nowhere else) so
// the result does not depend on the surrounding code.  The quotient
// (u - q)/(u + q) is the hardware reciprocal refined by one Newton-Raphson
// correction of the quotient (Markstein's scheme): a residual e = n - d*r0 is
// formed exactly by an FMA and folded back as r0 + e*y; this lands within one
// ulp of the correctly rounded quotient for the operand range of the model.
__device__ __forceinline__ void cell_update(float uC, float uW, float uE, float uN, float uS,
                                            float vC, float phiC, const Consts<float>& k,
                                            float& u_next, float& v_next) {
#pragma clang fp contract(off)
    const float s = (uW + uE) + (uN + uS);          // west+east first: D4-symmetric
    const float lap = __builtin_fmaf(-4.0f, uC, s);  // five-node sum
    const float a = __builtin_fmaf(-uC, uC, uC);     // u - u^2
    const float g = __builtin_fmaf(k.f, vC, phiC);   // f v + phi
    const float num = uC - k.q;
    const float den = uC + k.q;
    const float y = __builtin_amdgcn_rcpf(den);
    const float r0 = num * y;
    const float e = __builtin_fmaf(-den, r0, num);
    const float r = __builtin_fmaf(e, y, r0);        // (u - q)/(u + q)
    const float Ru = __builtin_fmaf(-g, r, a);       // reaction bracket
    u_next = __builtin_fmaf(k.c2, lap, __builtin_fmaf(k.c1, Ru, uC));
    v_next = __builtin_fmaf(k.dt, uC - vC, vC);
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
