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
// k0 = 1 + c1 - 4 c2, c1f = c1 f, omdt = 1 - dt and h2q = 1/(2q).
template <typename Real>
struct Consts {
    Real c1, c2, f, q, dt;
    Real k0, c1f, omdt, h2q;
};

// The constants of one parameter set (eps may be +inf: the reaction is then
// off, c1 = 0), every one formed in double and rounded once.
template <typename Real>
inline Consts<Real> make_consts(double eps, double f, double q, double D_u, double dt,
                                double dx) {
    const double c1 = dt / eps;
    const double c2 = dt * D_u / (dx * dx);
    Consts<Real> k;
    k.c1 = static_cast<Real>(c1);
    k.c2 = static_cast<Real>(c2);
    k.f = static_cast<Real>(f);
    k.q = static_cast<Real>(q);
    k.dt = static_cast<Real>(dt);
    k.k0 = static_cast<Real>(1.0 + c1 - 4.0 * c2);
    k.c1f = static_cast<Real>(c1 * f);
    k.omdt = static_cast<Real>(1.0 - dt);
    k.h2q = static_cast<Real>(1.0 / (2.0 * q));
    return k;
}

// FP32 update.  The forward-Euler step of Eq. (1),
//   u' = u + c1 [u - u^2 - (f v + phi)(u - q)/(u + q)] + c2 (s - 4u),
//   v' = v + dt (u - v),
// with (u - q)/(u + q) = 1 - 2q/(u + q), regrouped to take twelve
// instructions per cell (three adds of the five-node sum, eight FMA/mul and
// one hardware reciprocal, about 1 ulp):
//   G  = c1 f v + c1 phi                   (= c1 (f v + phi))
//   r  = 1 / ((u + q)/(2q))                (= 2q/(u + q); (u + q)/(2q) = u h2q + 1/2)
//   u' = u (k0 - c1 u) + (c2 s - G) + G r
//   v' = (1 - dt) v + dt u
// c1 phi arrives precomputed (`c1phi`, one FP32 multiply of the cell's phi).
// Contraction is pinned (fmaf where written, nowhere else), so every kernel
// that calls this gets bit-identical results.
__device__ __forceinline__ void cell_update(float uC, float uW, float uE, float uN, float uS,
                                            float vC, float c1phi, const Consts<float>& k,
                                            float& u_next, float& v_next) {
#pragma clang fp contract(off)
    const float s = (uE + uW) + (uS + uN);                         // west+east first: D4-symmetric
    const float G = __builtin_fmaf(k.c1f, vC, c1phi);              // c1 (f v + phi)
    const float r = __builtin_amdgcn_rcpf(__builtin_fmaf(uC, k.h2q, 0.5f));   // 2q / (u + q)
    const float x = __builtin_fmaf(k.c2, s, -G);                   // c2 s - G
    const float A = __builtin_fmaf(__builtin_fmaf(-k.c1, uC, k.k0), uC, x);
    u_next = __builtin_fmaf(G, r, A);
    v_next = __builtin_fmaf(k.omdt, vC, k.dt * uC);
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
