// reduce.hip -- whole-patch passes: primitive <-> conserved conversion
// (Sec. 3.5), the CFL rate reduction (eq. courantTimeStep) and the FP64
// conserved totals.
#include "hy_internal.h"
#include "hy_diag.h"

#include <math.h>

namespace hy {
namespace {

constexpr int RB = 256;  // threads per block for the flat passes

template <typename T> __device__ __forceinline__ T sqrt_(T x) { return sqrt(x); }

template <typename T>
__global__ void __launch_bounds__(RB) k_prim_to_cons(T *u, int64_t ncell, int64_t vs, int ndim, T inv_gm1)
{
    for (int64_t c = (int64_t)blockIdx.x * RB + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * RB) {
        const T rho = u[c];
        T ke = T(0);
        for (int d = 0; d < ndim; ++d) {
            const T v = u[c + (1 + d) * vs];
            ke += v * v;
            u[c + (1 + d) * vs] = rho * v;
        }
        const T p = u[c + (ndim + 1) * vs];
        u[c + (ndim + 1) * vs] = p * inv_gm1 + T(0.5) * rho * ke;
    }
}

template <typename T>
__global__ void __launch_bounds__(RB) k_cons_to_prim(const T *u, T *w, int64_t ncell, int64_t vs, int ndim, T gm1)
{
    for (int64_t c = (int64_t)blockIdx.x * RB + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * RB) {
        const T D = u[c];
        T s2 = T(0);
        w[c] = D;
        for (int d = 0; d < ndim; ++d) {
            const T s = u[c + (1 + d) * vs];
            s2 += s * s;
            w[c + (1 + d) * vs] = s / D;
        }
        w[c + (ndim + 1) * vs] = gm1 * (u[c + (ndim + 1) * vs] - T(0.5) * s2 / D);
    }
}

// max over cells and dimensions of (|v_q| + c) / dq; also latches bad states
template <typename T>
__global__ void __launch_bounds__(RB) k_cfl_rate(const T *u, int64_t ncell, int64_t vs, int ndim, T gamma, T gm1,
                                                 double idx0, double idx1, double idx2, DevCtl *ctl, int slot)
{
    double r = 0.0;
    bool bad = false;
    for (int64_t c = (int64_t)blockIdx.x * RB + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * RB) {
        const T D = u[c];
        T s2 = T(0);
        T v[3] = {T(0), T(0), T(0)};
        for (int d = 0; d < ndim; ++d) {
            const T s = u[c + (1 + d) * vs];
            s2 += s * s;
            v[d] = s / D;
        }
        const T p = gm1 * (u[c + (ndim + 1) * vs] - T(0.5) * s2 / D);
        bad |= !((D > T(0)) && (p > T(0)) && isfinite(D) && isfinite(p));  // positive and finite
        const T cs = sqrt_(gamma * p / D);
        const double id[3] = {idx0, idx1, idx2};
        for (int d = 0; d < ndim; ++d) r = fmax(r, ((double)fabs(v[d]) + (double)cs) * id[d]);
    }
    if (bad) atomicOr(&ctl->err, 1u);
    __shared__ double sr[RB / 64];
    for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off, 64));
    if ((threadIdx.x & 63) == 0) sr[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < RB / 64; ++w) m = fmax(m, sr[w]);
        if (m > 0.0) atomicMax(&ctl->rate[slot][blockIdx.x % RATE_SLOTS], (unsigned long long)__double_as_longlong(m));
    }
}

// Deterministic totals: block b sums the fixed chunk [b*C, (b+1)*C) of every
// variable in FP64 (per-thread strided partials, then a fixed LDS tree);
// a single block then adds the block partials in a fixed tree.
template <typename T>
__global__ void __launch_bounds__(RB) k_totals_partial(const T *u, int64_t ncell, int64_t vs, int nv, double *partials)
{
    __shared__ double red[RB];
    const int64_t C = (ncell + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * C;
    const int64_t end = beg + C < ncell ? beg + C : ncell;
    for (int v = 0; v < nv; ++v) {
        double s = 0.0;
        for (int64_t c = beg + threadIdx.x; c < end; c += RB) s += (double)u[c + v * vs];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = RB / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partials[v * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(RB) k_totals_final(const double *partials, int nblocks, int nv, int ndim, double dv,
                                                     DevCtl *ctl)
{
    __shared__ double red[RB];
    for (int v = 0; v < nv; ++v) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += RB) s += partials[v * nblocks + b];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = RB / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            // output order (D, Sx, Sy, Sz, G)
            const int slot = (v == 0) ? 0 : (v == nv - 1 ? 4 : v);
            ctl->totals[slot] = red[0] * dv;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = ndim; d < 3; ++d) ctl->totals[1 + d] = 0.0;
}

// Kinetic energy per component, sum over cells of D v_q^2 / 2 = S_q^2 / (2 D),
// in the same fixed chunks and trees as the totals (each cell's term formed
// in FP64 from the stored values); results in totals[5 + q].
template <typename T>
__global__ void __launch_bounds__(RB) k_kinetic_partial(const T *u, int64_t ncell, int64_t vs, int ndim,
                                                        double *partials)
{
    __shared__ double red[RB];
    const int64_t C = (ncell + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * C;
    const int64_t end = beg + C < ncell ? beg + C : ncell;
    for (int q = 0; q < ndim; ++q) {
        double s = 0.0;
        for (int64_t c = beg + threadIdx.x; c < end; c += RB) {
            const double S = (double)u[c + (1 + q) * vs];
            s += 0.5 * S * S / (double)u[c];
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = RB / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partials[q * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(RB) k_kinetic_final(const double *partials, int nblocks, int ndim, double dv,
                                                      DevCtl *ctl)
{
    __shared__ double red[RB];
    for (int q = 0; q < ndim; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += RB) s += partials[q * nblocks + b];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = RB / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) ctl->totals[5 + q] = red[0] * dv;
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = ndim; q < 3; ++q) ctl->totals[5 + q] = 0.0;
}

__global__ void k_ctl_reset_rate(DevCtl *ctl, int slot)
{
    if (threadIdx.x < RATE_SLOTS) ctl->rate[slot][threadIdx.x] = 0ull;
}

__global__ void k_ctl_init(DevCtl *ctl)
{
    ctl->time[0] = 0.0;
    ctl->time[1] = 0.0;
    for (int k = 0; k < RATE_SLOTS; ++k) {
        ctl->rate[0][k] = 0ull;
        ctl->rate[1][k] = 0ull;
    }
    ctl->err = 0u;
}

inline unsigned grid_for(int64_t n)
{
    int64_t g = (n + RB - 1) / RB;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

template <typename T>
hipError_t launch_prim_to_cons(T *u, int64_t ncell, int64_t vstride, int ndim, T gm1, T inv_gm1, hipStream_t s)
{
    (void)gm1;
    hipLaunchKernelGGL(k_prim_to_cons<T>, dim3(grid_for(ncell)), dim3(RB), 0, s, u, ncell, vstride, ndim, inv_gm1);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cons_to_prim(const T *u, T *w, int64_t ncell, int64_t vstride, int ndim, T gm1, hipStream_t s)
{
    hipLaunchKernelGGL(k_cons_to_prim<T>, dim3(grid_for(ncell)), dim3(RB), 0, s, u, w, ncell, vstride, ndim, gm1);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cfl_rate(const T *u, int64_t n0, int64_t n1, int64_t n2, int64_t vstride, int ndim, T gamma, T gm1,
                           const double *idx, DevCtl *ctl, int slot, hipStream_t s)
{
    const int64_t ncell = n0 * n1 * n2;
    hipLaunchKernelGGL(k_ctl_reset_rate, dim3(1), dim3(64), 0, s, ctl, slot);
    hipLaunchKernelGGL(k_cfl_rate<T>, dim3(grid_for(ncell)), dim3(RB), 0, s, u, ncell, vstride, ndim, gamma, gm1,
                       idx[0], idx[1], idx[2], ctl, slot);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_totals(const T *u, int64_t ncell, int64_t vstride, int ndim, double dv, double *partials,
                         int nblocks, DevCtl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_totals_partial<T>, dim3(nblocks), dim3(RB), 0, s, u, ncell, vstride, ndim + 2, partials);
    hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(RB), 0, s, partials, nblocks, ndim + 2, ndim, dv, ctl);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_kinetic(const T *u, int64_t ncell, int64_t vstride, int ndim, double dv, double *partials,
                          int nblocks, DevCtl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_kinetic_partial<T>, dim3(nblocks), dim3(RB), 0, s, u, ncell, vstride, ndim, partials);
    hipLaunchKernelGGL(k_kinetic_final, dim3(1), dim3(RB), 0, s, partials, nblocks, ndim, dv, ctl);
    return hipGetLastError();
}

hipError_t launch_ctl_reset_rate(DevCtl *ctl, int slot, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_reset_rate, dim3(1), dim3(64), 0, s, ctl, slot);
    return hipGetLastError();
}

hipError_t launch_ctl_init(DevCtl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(1), 0, s, ctl);
    return hipGetLastError();
}

#define HY_INST(T)                                                                                              \
    template hipError_t launch_prim_to_cons<T>(T *, int64_t, int64_t, int, T, T, hipStream_t);                  \
    template hipError_t launch_cons_to_prim<T>(const T *, T *, int64_t, int64_t, int, T, hipStream_t);          \
    template hipError_t launch_cfl_rate<T>(const T *, int64_t, int64_t, int64_t, int64_t, int, T, T,            \
                                           const double *, DevCtl *, int, hipStream_t);                         \
    template hipError_t launch_totals<T>(const T *, int64_t, int64_t, int, double, double *, int, DevCtl *,     \
                                         hipStream_t);                                                          \
    template hipError_t launch_kinetic<T>(const T *, int64_t, int64_t, int, double, double *, int, DevCtl *,    \
                                          hipStream_t);
HY_INST(float)
HY_INST(double)

}  // namespace hy
