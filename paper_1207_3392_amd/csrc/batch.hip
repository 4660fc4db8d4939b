// batch.hip -- many independent 1D patches ("tubes") advanced to a common end
// time in one persistent launch.
//
// Each workgroup pulls a tube index from a device-side atomic queue (tubes are
// listed in descending cost, so the longest tubes start first), holds the
// tube's primitives and face fluxes in LDS and its conserved state in
// registers, and runs the full single-level loop of Alg. 2 on it: dt =
// min(C dt_CFL, t_end - t) from a workgroup max-reduction (eq.
// courantTimeStep), then the two Runge-Kutta stages (eqs. RungeKutta1-3) of
// the same finite-volume update as the patch kernel (generalised minmod, HLL
// or HLLC, ghost cells by boundary kind).  When the queue is empty every
// workgroup exits.  The host captures the queue reset and this kernel in a
// hipGraph once and replays it.
#include "hy_batch.h"
#include "hy_internal.h"

#include <math.h>

namespace hy {
namespace {


__device__ __forceinline__ float rcpf_(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float soundf(float g, float p, float r)
{
    const float gp = g * p;
    return gp * __builtin_amdgcn_rsqf(gp * r);
}

// The generalised minmod slope of eq. MinMod divided by theta (see
// hy_face.h): MM(dm, (dm + dp) k, dp) = MM(MM(dm, dp), (dm + dp) k),
// k = 1 / (2 theta), the two-argument minmod being med3(x, y, 0); face
// values w +/- (theta / 2) slope.
__device__ __forceinline__ float slope_k(float wm, float w0, float wp, float k)
{
    const float dm = w0 - wm, dp = wp - w0;
    const float b = (dm + dp) * k;
    return __builtin_amdgcn_fmed3f(__builtin_amdgcn_fmed3f(dm, dp, 0.f), b, 0.f);
}

// 1D flux from primitive face states (rho, v, p); sg = sqrt(gamma)
__device__ __forceinline__ void flux1(const float (&wl)[3], const float (&wr)[3], float (&f)[3], float sg,
                                      float igm1, int solver)
{
    const float rl = wl[0], vl = wl[1], pl = wl[2];
    const float rr = wr[0], vr = wr[1], pr = wr[2];
    // sound speeds sg sqrt(p / rho), with sg folded into the signal speeds
    const float ul = pl * __builtin_amdgcn_rsqf(pl * rl), ur = pr * __builtin_amdgcn_rsqf(pr * rr);
    const float ap = fmaxf(0.f, fmaxf(sg * ul + vl, sg * ur + vr));
    const float am = fmaxf(0.f, fmaxf(sg * ul - vl, sg * ur - vr));
    if (solver == 0) {
        // HLL with each side's state entering once, as in hy_face.h:
        // F = cL U_L + cR U_R + wL P_L + wR P_R (P: p in the momentum, p v in
        // the energy), wL = a+ / (a+ + a-), wR = a- / (a+ + a-), cL = wL (v_L
        // + a-), cR = wR (v_R - a+); a+ + a- = 0 takes wL = wR = 1/2 (the
        // mean of the two fluxes)
        const float El = pl * igm1 + 0.5f * rl * vl * vl, Er = pr * igm1 + 0.5f * rr * vr * vr;
        const float den = ap + am;
        const bool pos = den > 0.f;
        const float inv = pos ? rcpf_(den) : 0.f;
        const float wL = pos ? ap * inv : 0.5f, wR = pos ? am * inv : 0.5f;
        const float cL = wL * (vl + am), cR = wR * (vr - ap);
        const float gL = cL * rl, gR = cR * rr;
        f[0] = gL + gR;
        f[1] = gL * vl + (gR * vr + (wL * pl + wR * pr));
        f[2] = cL * El + (cR * Er + (wL * (pl * vl) + wR * (pr * vr)));
        return;
    }
    // HLLC: Batten's middle speed, the middle state on the side K it selects
    // from the jump conditions across the s_K wave, and its physical flux
    // (equal to F_K + s_K (U*_K - U_K)); supersonic: middle speed v_K, so the
    // middle state is U_K and the flux F_K
    const float ql = am + vl, qr = ap - vr;
    const float A = rr * qr, B = rl * ql;
    const float a_m = (A * vr + (B * vl + (pl - pr))) * rcpf_(A + B);
    const bool sup = (am == 0.f) | (ap == 0.f);
    const bool useL = (am == 0.f) | ((ap != 0.f) & (a_m >= 0.f));
    const float rK = useL ? rl : rr, vK = useL ? vl : vr, pK = useL ? pl : pr;
    const float sK = useL ? -am : ap;
    const float sm = sup ? vK : a_m;
    const float EK = pK * igm1 + 0.5f * rK * vK * vK;
    const float qk = sK - vK;
    const float rq = rK * qk;
    const float ps = pK + rq * (sm - vK);
    // (E* + p*) sm = (q_K E_K - p_K v_K + p* s_K) sm / (s_K - sm), as in hy_face.h
    const float ism = rcpf_(sK - sm) * sm;
    const float fd = rq * ism;
    f[0] = fd;
    f[1] = fd * sm + ps;
    f[2] = (qk * EK - pK * vK + ps * sK) * ism;
}

__global__ void k_batch_reset(BatchCtl *ctl)
{
    ctl->next = 0u;
}

// BT threads per workgroup, CPT cells per thread (BT * CPT >= the batch's
// longest tube; the smaller CPT that fits keeps the state in fewer registers)
template <int BT, int CPT>
__global__ void __launch_bounds__(BT) k_batch(const TubeDesc *__restrict__ tubes, const int *__restrict__ order,
                                              float *__restrict__ U, int64_t ntot, BatchCtl *ctl,
                                              TubeStatus *__restrict__ status, int ntubes, int nmax)
{
    extern __shared__ float lds[];
    float *sW = lds;                   // 3 x (nmax + 4): primitives with 2 ghost cells each side
    float *sF = lds + 3 * (nmax + 4);  // 3 x (nmax + 1): face fluxes
    __shared__ float sred[BT / 64];
    __shared__ int sidx;
    const int tid = threadIdx.x;
    const int SW = nmax + 4, SF = nmax + 1;
    const double t_end = ctl->t_end, cfl = ctl->cfl;
    const int solver = ctl->solver;
    const int max_steps = ctl->max_steps;

    for (;;) {
        if (tid == 0) sidx = (int)atomicAdd(&ctl->next, 1u);
        __syncthreads();
        const int q = sidx;
        __syncthreads();
        if (q >= ntubes) break;
        const int ti = order[q];
        const TubeDesc d = tubes[ti];
        const int n = d.n;
        const float g = d.gamma, gm1 = d.gamma - 1.f, igm1 = 1.f / (d.gamma - 1.f);
        const float sg = sqrtf(d.gamma), lk = 0.5f / d.theta, hs = 0.5f * d.theta;
        const float idx = d.idx;

        // conserved state of the owned cells (cell i = tid + k * BT)
        float U0[CPT][3], Us[CPT][3];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int i = tid + k * BT;
#pragma unroll
            for (int v = 0; v < 3; ++v) U0[k][v] = i < n ? U[v * ntot + d.off + i] : 1.f;
        }

        bool bad = false;
        // stage input -> primitives in LDS, the ghosts written by the threads
        // that own their source cells (one barrier); with want_rate the
        // block max of (|v| + c) / dx of the state is returned (each wave's
        // max goes to LDS before the barrier)
        auto fill = [&](const float (&S)[CPT][3], bool want_rate) -> float {
            float rate = 0.f;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int i = tid + k * BT;
                if (i < n) {
                    const float D = S[k][0], ir = rcpf_(D);
                    const float v = S[k][1] * ir;
                    const float p = gm1 * (S[k][2] - 0.5f * S[k][1] * v);
                    // rho and p positive and finite (one class test each)
                    bad |= !(__builtin_amdgcn_classf(D, 0x180) & __builtin_amdgcn_classf(p, 0x180));
                    sW[0 * SW + i + 2] = D;
                    sW[1 * SW + i + 2] = v;
                    sW[2 * SW + i + 2] = p;
                    if (want_rate) rate = fmaxf(rate, (fabsf(v) + soundf(g, p, D)) * idx);
                    if (i < 2 || i >= n - 2) {
                        // ghosts -2, -1, n, n+1 whose source is this cell
#pragma unroll
                        for (int gk = 0; gk < 4; ++gk) {
                            const int gi = gk < 2 ? gk - 2 : n + gk - 2;
                            const int bc = gk < 2 ? d.bclo : d.bchi;
                            int src;
                            bool flip = false;
                            if (bc == BC_PERIODIC) src = gk < 2 ? gi + n : gi - n;
                            else if (bc == BC_OUTFLOW) src = gk < 2 ? 0 : n - 1;
                            else { src = gk < 2 ? -1 - gi : 2 * n - 1 - gi; flip = true; }
                            if (src == i) {
                                sW[0 * SW + gi + 2] = D;
                                sW[1 * SW + gi + 2] = flip ? -v : v;
                                sW[2 * SW + gi + 2] = p;
                            }
                        }
                    }
                }
            }
            if (want_rate) {
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) rate = fmaxf(rate, __shfl_xor(rate, off, 64));
                if ((tid & 63) == 0) sred[tid >> 6] = rate;
            }
            __syncthreads();
            float m = 0.f;
            if (want_rate) {
#pragma unroll
                for (int w = 0; w < BT / 64; ++w) m = fmaxf(m, sred[w]);
            }
            return m;
        };
        auto faces = [&]() {
            for (int f = tid; f <= n; f += BT) {
                float wl[3], wr[3], fl[3];
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    const float *w = sW + v * SW + f;  // w[0..3] = cells f-2 .. f+1
                    wl[v] = w[1] + hs * slope_k(w[0], w[1], w[2], lk);
                    wr[v] = w[2] - hs * slope_k(w[1], w[2], w[3], lk);
                }
                flux1(wl, wr, fl, sg, igm1, solver);
#pragma unroll
                for (int v = 0; v < 3; ++v) sF[v * SF + f] = fl[v];
            }
            __syncthreads();
        };

        double t = 0.0;
        int steps = 0;
        float r = fill(U0, true);  // CFL rate of the state
        bool stop = false;
        while (t < t_end && !stop) {
            double dt = fmin(cfl / (double)r, t_end - t);
            if (!(dt > 0.0) || steps >= max_steps) {  // non-finite rate or step cap: stop this tube
                stop = true;
                break;
            }
            const float dtf = (float)dt;
            // the step's weight of a face-flux difference, per stage
            const float c1 = dtf * idx, c2 = 0.5f * c1;
            // stage 1: U1 = U^n + dt L(U^n); the primitives of U^n are in LDS
            faces();
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int i = tid + k * BT;
#pragma unroll
                for (int v = 0; v < 3; ++v)
                    Us[k][v] = i < n ? U0[k][v] + c1 * (sF[v * SF + i] - sF[v * SF + i + 1]) : 1.f;
            }
            // (no barrier: the flux reads above end before any thread passes
            // the barrier in fill, and only the next faces() writes sF)
            fill(Us, false);
            // stage 2: U^{n+1} = (U^n + U1 + dt L(U1)) / 2
            faces();
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int i = tid + k * BT;
#pragma unroll
                for (int v = 0; v < 3; ++v)
                    U0[k][v] = i < n ? 0.5f * (U0[k][v] + Us[k][v]) + c2 * (sF[v * SF + i] - sF[v * SF + i + 1])
                                     : 1.f;
            }
            r = fill(U0, true);
            t += dt;
            ++steps;
        }
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int i = tid + k * BT;
            if (i < n)
#pragma unroll
                for (int v = 0; v < 3; ++v) U[v * ntot + d.off + i] = U0[k][v];
        }
        // per-tube status: any thread's bad flag, steps and time reached
        __shared__ int sbad;
        if (tid == 0) sbad = 0;
        __syncthreads();
        if (bad) atomicOr(&sbad, 1);
        __syncthreads();
        if (tid == 0) {
            status[ti].steps = steps;
            status[ti].err = sbad | (stop ? 2 : 0);
            status[ti].t = t;
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_batch_reset(BatchCtl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, ctl);
    return hipGetLastError();
}

namespace {
// Two register footprints per workgroup size: tubes up to 4096 cells, or up
// to BATCH_NMAX (6144).
constexpr int SMALL_NMAX = 4096;

template <int BT>
const void *batch_kernel_bt(int nmax)
{
    if (nmax <= SMALL_NMAX) return (const void *)k_batch<BT, SMALL_NMAX / BT>;
    return (const void *)k_batch<BT, BATCH_NMAX / BT>;
}

const void *batch_kernel(int bt, int nmax)
{
    switch (bt) {
    case 256: return batch_kernel_bt<256>(nmax);
    case 512: return batch_kernel_bt<512>(nmax);
    default: return batch_kernel_bt<1024>(nmax);
    }
}
}  // namespace

bool batch_bt_supported(int bt) { return bt == 256 || bt == 512 || bt == 1024; }

hipError_t prepare_batch(int nmax)
{
    // dynamic LDS above the 64 KiB default must be allowed explicitly
    hipError_t e = hipSuccess;
    for (int bt : {256, 512, 1024})
        if (e == hipSuccess)
            e = hipFuncSetAttribute(batch_kernel(bt, nmax), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)batch_lds_bytes(nmax));
    return e;
}

hipError_t launch_batch(const TubeDesc *tubes, const int *order, float *U, int64_t ntot, BatchCtl *ctl,
                        TubeStatus *status, int ntubes, int nmax, int nblocks, int bt, hipStream_t s)
{
    if (nmax < 1 || nmax > BATCH_NMAX || !batch_bt_supported(bt)) return hipErrorInvalidValue;
    const size_t lds = batch_lds_bytes(nmax);
    void *args[] = {(void *)&tubes, (void *)&order, (void *)&U, (void *)&ntot, (void *)&ctl,
                    (void *)&status, (void *)&ntubes, (void *)&nmax};
    const hipError_t e = hipLaunchKernel(batch_kernel(bt, nmax), dim3(nblocks), dim3(bt), args, lds, s);
    return e != hipSuccess ? e : hipGetLastError();
}

size_t batch_lds_bytes(int nmax) { return sizeof(float) * (3 * (size_t)(nmax + 4) + 3 * (size_t)(nmax + 1)); }

int batch_blocks_per_cu(int nmax, int bt)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel(bt, nmax), bt, batch_lds_bytes(nmax)) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

}  // namespace hy
