// Pointwise device math of the finite-volume update, shared by the stage
// kernels and the multilevel kernels so that both compute the same face
// fluxes: primitive recovery (Sec. 3.5), the generalised-minmod slope (eq.
// MinMod) and the HLL / HLLC fluxes (eqs. FluxHLL, FluxHLLC and the middle
// wave of eq. MiddleWaveSpeed).  Internal; every user gets its own copy.
#pragma once

#include "hy_internal.h"

#include <math.h>

namespace hy {
namespace {

// ---------------------------------------------------------------- math ----

template <typename T> __device__ __forceinline__ T rcp_(T x);
template <> __device__ __forceinline__ float rcp_<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp_<double>(double x) { return 1.0 / x; }

// sqrt(p / rho), the sound speed divided by sqrt(gamma), evaluated as
// p rsqrt(p rho); the solvers fold sqrt(gamma) into the signal speeds
template <typename T> __device__ __forceinline__ T sound1_(T p, T rho);
template <> __device__ __forceinline__ float sound1_<float>(float p, float r)
{
    return p * __builtin_amdgcn_rsqf(p * r);
}
template <> __device__ __forceinline__ double sound1_<double>(double p, double r) { return sqrt(p / r); }

// c_s = sqrt(gamma p / rho), evaluated as (gamma p) rsqrt(gamma p rho)
template <typename T> __device__ __forceinline__ T sound_(T gamma, T p, T rho);
template <> __device__ __forceinline__ float sound_<float>(float g, float p, float r)
{
    float gp = g * p;
    return gp * __builtin_amdgcn_rsqf(gp * r);
}
template <> __device__ __forceinline__ double sound_<double>(double g, double p, double r)
{
    return sqrt(g * p / r);
}

template <typename T> __device__ __forceinline__ T max3_(T a, T b, T c) { return fmax(a, fmax(b, c)); }

// ------------------------------------------------------ fluid variables ----

// x > 0 and finite: one class test in FP32 (positive normal or subnormal)
template <typename T> __device__ __forceinline__ bool pos_finite(T x);
template <> __device__ __forceinline__ bool pos_finite<float>(float x) { return __builtin_amdgcn_classf(x, 0x180); }
template <> __device__ __forceinline__ bool pos_finite<double>(double x)
{
    return __builtin_amdgcn_class(x, 0x180);
}

// primitives (rho, v, p) from conserved (D, S, G), m = 1; returns false on
// rho <= 0, p <= 0 or a non-finite value
template <int ND, typename T>
__device__ __forceinline__ bool to_prim(const T (&u)[ND + 2], T (&w)[ND + 2], T gm1)
{
    const T ir = rcp_(u[0]);
    T ke = T(0);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        w[1 + d] = u[1 + d] * ir;
        ke += u[1 + d] * w[1 + d];
    }
    w[0] = u[0];
    w[ND + 1] = gm1 * (u[ND + 1] - T(0.5) * ke);
    return pos_finite(w[0]) & pos_finite(w[ND + 1]);
}

template <typename T> __device__ __forceinline__ T med3_(T a, T b, T c);
template <> __device__ __forceinline__ float med3_<float>(float a, float b, float c)
{
    return __builtin_amdgcn_fmed3f(a, b, c);
}
template <> __device__ __forceinline__ double med3_<double>(double a, double b, double c)
{
    return fmax(fmin(a, b), fmin(fmax(a, b), c));
}

// Twice the generalised-minmod slope of eq. MinMod as a per-cell difference:
// with a = 2 theta dm, b = dm + dp, c = 2 theta dp, MM(a, b, c) (the argument
// of least magnitude when all share a sign, else 0) = 2 MM(theta dm,
// (dm + dp) / 2, theta dp) exactly, evaluated as MM(MM(a, c), b) (b shares
// the sign of a and c when they agree; see slope_mm).  Face values are then
// w +/- slope / 4.
template <typename T>
__device__ __forceinline__ T slope2_mm(T wm, T w0, T wp, T theta2)
{
    const T dm = w0 - wm, dp = wp - w0;
    const T a = theta2 * dm, b = dm + dp, c = theta2 * dp;
    return med3_(med3_(a, c, T(0)), b, T(0));
}

// The generalised-minmod slope of eq. MinMod divided by theta: scaling every
// argument of MM by 1 / theta (a positive factor commutes with MM) gives
// MM(dm, (dm + dp) k, dp) with k = 1 / (2 theta); the face values are then
// w +/- hs * slope with hs = theta / 2.  The factors theta leave the per-cell
// work this way.  The middle argument b = (dm + dp) k carries the sign of
// dm and dp whenever those two agree, so MM(dm, b, dp) = MM(MM(dm, dp), b),
// and the two-argument minmod is med3(x, y, 0) (the argument nearer to zero
// when they share a sign, else 0): two median instructions, the same value
// as med3(min3, max3, 0) bit for bit (each form selects one of its inputs).
template <typename T>
__device__ __forceinline__ T slope_mm(T wm, T w0, T wp, T k)
{
    const T dm = w0 - wm, dp = wp - w0;
    const T b = (dm + dp) * k;
    return med3_(med3_(dm, dp, T(0)), b, T(0));
}

// The per-patch constants of slope_mm and of the face values, formed the
// same way by every kernel that computes a face flux of the same state.
template <typename T> struct ThetaLim {
    T k, hs;
};
template <typename T> __device__ __forceinline__ ThetaLim<T> theta_lim(T theta)
{
    return ThetaLim<T>{T(0.5) / theta, T(0.5) * theta};
}

// ------------------------------------------------------ Riemann solvers ----

// Flux normal to Q from the primitive face states wl (left), wr (right).
// sg = sqrt(gamma) (formed once per kernel by the caller, the same way
// everywhere: sqrt_gamma below).
template <int ND, int Q, int SOLVER, typename T>
__device__ __forceinline__ void riemann(const T (&wl)[ND + 2], const T (&wr)[ND + 2], T (&f)[ND + 2],
                                        T sg, T inv_gm1)
{
    constexpr int IP = ND + 1;
    const T rl = wl[0], vl = wl[1 + Q], pl = wl[IP];
    const T rr = wr[0], vr = wr[1 + Q], pr = wr[IP];
    const T ul = sound1_(pl, rl), ur = sound1_(pr, rr);
    // outer speed estimates alpha_+/- = max(0, +/-lambda_+/-(L), +/-lambda_+/-(R)),
    // c = sg u
    const T ap = max3_(T(0), sg * ul + vl, sg * ur + vr);
    const T am = max3_(T(0), sg * ul - vl, sg * ur - vr);
    if constexpr (SOLVER == 0) {
        T kl = T(0), kr = T(0);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            kl += wl[1 + d] * wl[1 + d];
            kr += wr[1 + d] * wr[1 + d];
        }
        const T El = pl * inv_gm1 + T(0.5) * rl * kl;
        const T Er = pr * inv_gm1 + T(0.5) * rr * kr;
        // F = (a+ F_L + a- F_R - a+ a- (U_R - U_L)) / (a+ + a-).  With the
        // physical flux F = v U + P (P: p in the normal momentum, p v in the
        // energy) each side's state enters once:
        //   F = cL U_L + cR U_R + wL P_L + wR P_R,
        //   wL = a+ / (a+ + a-), wR = a- / (a+ + a-),
        //   cL = wL (v_L + a-), cR = wR (v_R - a+).
        // a+ + a- = 0 (both sides at rest with c = 0, so a+ = a- = 0) takes
        // wL = wR = 1/2, which makes the same coefficients the mean of the
        // two fluxes.
        const T den = ap + am;
        const bool pos = den > T(0);
        const T inv = pos ? rcp_(den) : T(0);
        const T wL = pos ? ap * inv : T(0.5), wR = pos ? am * inv : T(0.5);
        const T cL = wL * (vl + am), cR = wR * (vr - ap);
        const T gL = cL * rl, gR = cR * rr;  // the coefficients of the velocities in the momentum
        f[0] = gL + gR;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            if (d == Q) f[1 + d] = gL * wl[1 + d] + (gR * wr[1 + d] + (wL * pl + wR * pr));
            else f[1 + d] = gL * wl[1 + d] + gR * wr[1 + d];
        }
        f[IP] = cL * El + (cR * Er + (wL * (pl * vl) + wR * (pr * vr)));
    } else {
        // Batten's middle-wave speed (eq. MiddleWaveSpeed):
        // (A v_R + B v_L + p_L - p_R) / (A + B), A = rho_R (a+ - v_R), B = rho_L (a- + v_L)
        const T ql = am + vl, qr = ap - vr;
        const T A = rr * qr, B = rl * ql;
        const T am_ = (A * vr + (B * vl + (pl - pr))) * rcp_(A + B);
        // eq. FluxHLLC: alpha_- = 0 selects L, then alpha_+ = 0 selects R,
        // then the sign of alpha_m selects the middle state on its side
        const bool sup = (am == T(0)) | (ap == T(0));
        const bool useL = (am == T(0)) | ((ap != T(0)) & (am_ >= T(0)));
        T wk[ND + 2];
#pragma unroll
        for (int v = 0; v < ND + 2; ++v) wk[v] = useL ? wl[v] : wr[v];
        const T sK = useL ? -am : ap;
        const T rK = wk[0], vK = wk[1 + Q], pK = wk[IP];
        // supersonic (s_K = 0): a middle speed equal to v_K makes the middle
        // state U_K itself, so the flux below is F_K
        const T sm = sup ? vK : am_;
        T kk = T(0);
#pragma unroll
        for (int d = 0; d < ND; ++d) kk += wk[1 + d] * wk[1 + d];
        const T EK = pK * inv_gm1 + T(0.5) * rK * kk;
        // middle state from the jump conditions across the K-side outer wave
        // (s_K - sm is nonzero: opposite signs, or v_K != 0 when supersonic):
        // rho* = rho_K q_K / (s_K - sm), p* = p_K + rho_K q_K (sm - v_K),
        // E* = (q_K E_K - p_K v_K + p* sm) / (s_K - sm), q_K = s_K - v_K
        const T qk = sK - vK;
        const T rq = rK * qk;
        const T ps = pK + rq * (sm - vK);
        // F_K + s_K (U*_K - U_K) equals the physical flux of the middle state
        // (the jump conditions across the s_K wave), formed directly: mass
        // flux rho* sm, and energy flux (E* + p*) sm = (q_K E_K - p_K v_K +
        // p* s_K) sm / (s_K - sm) (the p* sm terms cancel)
        const T ism = rcp_(sK - sm) * sm;
        const T fd = rq * ism;
        f[0] = fd;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            if (d == Q) f[1 + d] = fd * sm + ps;
            else f[1 + d] = fd * wk[1 + d];
        }
        f[IP] = (qk * EK - pK * vK + ps * sK) * ism;
    }
}

// Face flux for the kernel's solver: the HLLC switch takes HLL where hll is
// set (a shock flagged along a direction transverse to this face), HLLC
// elsewhere; the other solvers ignore hll.
template <int ND, int Q, int SOLVER, typename T>
__device__ __forceinline__ void face_flux(const T (&wl)[ND + 2], const T (&wr)[ND + 2], T (&f)[ND + 2], T sg,
                                          T inv_gm1, bool hll)
{
    if constexpr (SOLVER == SOLVER_HLLC_SWITCH) {
        if (hll) riemann<ND, Q, SOLVER_HLL>(wl, wr, f, sg, inv_gm1);
        else riemann<ND, Q, SOLVER_HLLC>(wl, wr, f, sg, inv_gm1);
    } else {
        (void)hll;
        riemann<ND, Q, SOLVER>(wl, wr, f, sg, inv_gm1);
    }
}

template <typename T> __device__ __forceinline__ T sqrt_gamma(T gamma) { return sqrt(gamma); }

// ------------------------------------------------ box face fluxes ----

__device__ __forceinline__ int64_t at(const Grid &g, int i, int j, int k)
{
    return ((int64_t)k * g.m[1] + j) * g.m[0] + i;
}

template <int ND, typename T>
__device__ __forceinline__ void load_prim(const T *u, const Grid &g, int64_t c, T gm1, T (&w)[ND + 2])
{
    T uu[ND + 2];
#pragma unroll
    for (int v = 0; v < ND + 2; ++v) uu[v] = u[v * g.vs + c];
    (void)to_prim<ND>(uu, w, gm1);
}

// The faces of one box normal to Q on one side (0: low, 1: high): one
// thread per face position transverse to Q.
template <int ND, int Q, int SOLVER, typename T>
__device__ __forceinline__ void box_faces(const T *u, const Grid &g, const Box &b, int t, int side, T gamma, T gm1,
                                          T inv_gm1, T theta, double w, bool assign, double *acc_lo, double *acc_hi)
{
    constexpr int R1 = Q == 0 ? 1 : 0, R2 = Q == 2 ? 1 : 2;  // transverse dimensions, the lower one fastest
    const int faces = b.n[R1] * b.n[R2];
    if (t >= faces) return;
    const int t1 = t % b.n[R1], t2 = t / b.n[R1];
    {
        const int f = side == 0 ? b.lo[Q] : b.lo[Q] + b.n[Q];  // face between cells f - 1 and f
        T w4[4][ND + 2];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            int c3[3];
            c3[Q] = f - 2 + s;
            c3[R1] = b.lo[R1] + t1;
            c3[R2] = b.lo[R2] + t2;
            load_prim<ND>(u, g, at(g, c3[0], c3[1], c3[2]), gm1, w4[s]);
        }
        T wl[ND + 2], wr[ND + 2], fl[ND + 2];
        const ThetaLim<T> lim = theta_lim(theta);
#pragma unroll
        for (int v = 0; v < ND + 2; ++v) {
            wl[v] = w4[1][v] + lim.hs * slope_mm(w4[0][v], w4[1][v], w4[2][v], lim.k);
            wr[v] = w4[2][v] - lim.hs * slope_mm(w4[1][v], w4[2][v], w4[3][v], lim.k);
        }
        face_flux<ND, Q, SOLVER>(wl, wr, fl, sqrt_gamma(gamma), inv_gm1, false);
        double *acc = side == 0 ? acc_lo : acc_hi;
#pragma unroll
        for (int v = 0; v < ND + 2; ++v) {
            double &a = acc[(int64_t)v * faces + t];
            a = (assign ? 0.0 : a) + w * (double)fl[v];
        }
    }
}

}  // namespace
}  // namespace hy
