// fmr.hip -- kernels of fixed multilevel refinement (Sec. 2, prolongation and
// restriction; Sec. 3.6, Algs. EvolveLevel and StepLevel): the exterior of a
// refined level by prolongation, the boundary fluxes a level hands to its
// parent and the fluxes the parent computed at the same faces, the
// coarse/fine flux replacement, restriction, and the CFL rate and conserved
// totals over part of an array.  These are thin passes over faces or over a
// level's two-cell shell; the cell update itself is the stage kernel's
// (in its padded mode on refined levels).
#include "hy_fmr.h"
#include "hy_face.h"
#include "hy_ride.h"

#include <algorithm>

namespace hy {
namespace {

constexpr int FB = 64;   // threads per block of the shell and face kernels
constexpr int TB = 256;  // threads per block of the reductions

constexpr int SB = 256;  // threads per block of the exterior-shell kernels

template <int ND, typename T>
__global__ void __launch_bounds__(SB) k_prolong(RideJob<T> j)
{
    ride_run<ND>(j, blockIdx.x, threadIdx.x, SB);
}

// Up to two boxes of one array in one launch: blockIdx.y = (box * ND + Q) * 2
// + side.
// assign[k]: box k's accumulators are overwritten, not added to.
struct FluxSet {
    Box b[2];
    double *acc[2][3][2];
    int assign[2];
};

template <int ND, int SOLVER, typename T>
__global__ void __launch_bounds__(FB) k_box_flux(const T *u, Grid g, FluxSet fs, T gamma, T gm1, T inv_gm1, T theta,
                                                  const double *dt)
{
    const double w = 0.5 * *dt;
    const int side = blockIdx.y & 1, bq = blockIdx.y >> 1;
    const int bx = bq / ND, q = bq - bx * ND;
    const int t = blockIdx.x * FB + threadIdx.x;
    const Box &b = fs.b[bx];
    if (q == 0)
        box_faces<ND, 0, SOLVER>(u, g, b, t, side, gamma, gm1, inv_gm1, theta, w, fs.assign[bx] != 0,
                                     fs.acc[bx][0][0], fs.acc[bx][0][1]);
    if constexpr (ND >= 2)
        if (q == 1)
            box_faces<ND, 1, SOLVER>(u, g, b, t, side, gamma, gm1, inv_gm1, theta, w, fs.assign[bx] != 0,
                                     fs.acc[bx][1][0], fs.acc[bx][1][1]);
    if constexpr (ND >= 3)
        if (q == 2)
            box_faces<ND, 2, SOLVER>(u, g, b, t, side, gamma, gm1, inv_gm1, theta, w, fs.assign[bx] != 0,
                                     fs.acc[bx][2][0], fs.acc[bx][2][1]);
}

// One thread per coarse face of the child box normal to Q (both sides).
template <int ND, int Q, typename T>
__device__ __forceinline__ void reflux_faces(T *u, const Grid &g, const Box &b, int t, const double *c_lo,
                                             const double *c_hi, const double *f_lo, const double *f_hi, double idq)
{
    constexpr int R1 = Q == 0 ? 1 : 0, R2 = Q == 2 ? 1 : 2;  // transverse dimensions, the lower one fastest
    constexpr int A1 = R1 < ND ? 2 : 1, A2 = R2 < ND ? 2 : 1;
    const int faces = b.n[R1] * b.n[R2];
    const int ffaces = faces * A1 * A2, fn1 = b.n[R1] * A1;
    if (t >= faces) return;
    const int t1 = t % b.n[R1], t2 = t / b.n[R1];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const double *cf = side == 0 ? c_lo : c_hi;
        const double *ff = side == 0 ? f_lo : f_hi;
        int c3[3];
        c3[Q] = side == 0 ? b.lo[Q] - 1 : b.lo[Q] + b.n[Q];
        c3[R1] = b.lo[R1] + t1;
        c3[R2] = b.lo[R2] + t2;
        const int64_t c = at(g, c3[0], c3[1], c3[2]);
#pragma unroll
        for (int v = 0; v < ND + 2; ++v) {
            double sum = 0.0;
#pragma unroll
            for (int o2 = 0; o2 < A2; ++o2)
#pragma unroll
                for (int o1 = 0; o1 < A1; ++o1)
                    sum += ff[(int64_t)v * ffaces + (A2 * t2 + o2) * fn1 + A1 * t1 + o1];
            const double phi_f = sum / (double)(A1 * A2);
            const double phi_c = cf[(int64_t)v * faces + t];
            const double corr = side == 0 ? phi_c - phi_f : phi_f - phi_c;
            T &x = u[v * g.vs + c];
            x = (T)((double)x + corr * idq);
        }
    }
}

struct RefluxSet {
    const double *c[3][2];
    const double *f[3][2];
    double idq[3];
};

// Every parent cell of b (interior cell i, j, k) becomes the mean of its 2^ND
// children, the child being a padded level (interior at offset NG).
template <int ND, typename T>
__device__ __forceinline__ void restrict_cell(T *parent, const Grid &pg, const Box &b, const T *child, const Grid &cg,
                                              int i, int j, int k)
{
    const int64_t pc = at(pg, b.lo[0] + i, b.lo[1] + j, b.lo[2] + k);
    constexpr int NC = 1 << ND;
#pragma unroll
    for (int v = 0; v < ND + 2; ++v) {
        double sum = 0.0;
#pragma unroll
        for (int o = 0; o < NC; ++o) {
            const int ci = FMR_NG + 2 * i + (o & 1);
            const int cj = ND > 1 ? FMR_NG + 2 * j + ((o >> 1) & 1) : 0;
            const int ck = ND > 2 ? FMR_NG + 2 * k + ((o >> 2) & 1) : 0;
            sum += (double)child[v * cg.vs + at(cg, ci, cj, ck)];
        }
        parent[v * pg.vs + pc] = (T)(sum / (double)NC);
    }
}

// The replacement and the restriction of one child box in one launch: the
// first ND * rblocks blocks correct the cells just outside the box (rblocks
// blocks per dimension Q), the rest restrict the cells under it, x fastest.
// The two sets of cells are disjoint, and neither reads what the other writes.
template <int ND, typename T>
__global__ void __launch_bounds__(FB) k_reflux_restrict(T *u, Grid g, Box b, RefluxSet r, const T *child, Grid cg,
                                                        int rblocks, int rcblocks, RideJob<T> ride)
{
    const int bid = blockIdx.x;
    if (bid >= rcblocks) {  // a job riding on the launch
        ride_run<ND>(ride, bid - rcblocks, threadIdx.x, FB);
        return;
    }
    if (bid < ND * rblocks) {
        const int q = bid / rblocks, t = (bid - q * rblocks) * FB + threadIdx.x;
        if (q == 0) reflux_faces<ND, 0>(u, g, b, t, r.c[0][0], r.c[0][1], r.f[0][0], r.f[0][1], r.idq[0]);
        if constexpr (ND >= 2)
            if (q == 1) reflux_faces<ND, 1>(u, g, b, t, r.c[1][0], r.c[1][1], r.f[1][0], r.f[1][1], r.idq[1]);
        if constexpr (ND >= 3)
            if (q == 2) reflux_faces<ND, 2>(u, g, b, t, r.c[2][0], r.c[2][1], r.f[2][0], r.f[2][1], r.idq[2]);
        return;
    }
    const int64_t cell = (int64_t)(bid - ND * rblocks) * FB + threadIdx.x;
    const int64_t nxy = (int64_t)b.n[0] * b.n[1];
    if (cell >= nxy * b.n[2]) return;
    const int k = (int)(cell / nxy);
    const int rem = (int)(cell - (int64_t)k * nxy);
    const int j = rem / b.n[0], i = rem - j * b.n[0];
    restrict_cell<ND>(u, g, b, child, cg, i, j, k);
}

// Grid-stride over the box's cells; one atomic per block.
template <int ND, typename T>
__global__ void __launch_bounds__(TB) k_box_rate(const T *u, Grid g, Box b, T gamma, T gm1, double idq0, double idq1,
                                                  double idq2, unsigned long long *rate_bits)
{
    __shared__ double red[TB];
    const double idq[3] = {idq0, idq1, idq2};
    const int nx = b.n[0], nxy = b.n[0] * b.n[1], cells = nxy * b.n[2];
    double m = 0.0;
    for (int c = blockIdx.x * TB + threadIdx.x; c < cells; c += gridDim.x * TB) {
        const int k = c / nxy, r = c - k * nxy, j = r / nx, i = r - j * nx;
        T w[ND + 2];
        load_prim<ND>(u, g, at(g, b.lo[0] + i, b.lo[1] + j, b.lo[2] + k), gm1, w);
        const double cs = (double)sound_(gamma, w[ND + 1], w[0]);
#pragma unroll
        for (int q = 0; q < ND; ++q) m = fmax(m, (fabs((double)w[1 + q]) + cs) * idq[q]);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = TB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicMax(&rate_bits[blockIdx.x % FMR_RATE_SLOTS], (unsigned long long)__double_as_longlong(red[0]));
}

template <int ND, typename T>
__global__ void __launch_bounds__(TB) k_leaf_totals(const T *u, Grid g, Box b, Box hole, double dv, double *partials)
{
    __shared__ double red[TB];
    const int j = blockIdx.x, k = blockIdx.y;
    const int row = k * b.n[1] + j;
    const int y = b.lo[1] + j, z = b.lo[2] + k;
    const bool row_in_hole = hole.n[0] > 0 && y >= hole.lo[1] && y < hole.lo[1] + hole.n[1] && z >= hole.lo[2] &&
                             z < hole.lo[2] + hole.n[2];
    double s[ND + 2];
#pragma unroll
    for (int v = 0; v < ND + 2; ++v) s[v] = 0.0;
    for (int i = threadIdx.x; i < b.n[0]; i += TB) {
        const int x = b.lo[0] + i;
        if (row_in_hole && x >= hole.lo[0] && x < hole.lo[0] + hole.n[0]) continue;
        const int64_t c = at(g, x, y, z);
#pragma unroll
        for (int v = 0; v < ND + 2; ++v) s[v] += (double)u[v * g.vs + c];
    }
#pragma unroll
    for (int v = 0; v < ND + 2; ++v) {
        red[threadIdx.x] = s[v];
        __syncthreads();
        for (int st = TB / 2; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int slot = v == 0 ? 0 : (v == ND + 1 ? 4 : v);
            partials[row * 5 + slot] = red[0] * dv;
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) {
        // slots of absent momentum components
        const int slot = threadIdx.x;
        if (slot > ND && slot < 4) partials[row * 5 + slot] = 0.0;
    }
}

template <int ND, typename T>
hipError_t box_flux_nd(const T *u, const Grid &g, const FluxSet &fs, int nbox, int solver, T gamma, T gm1, T inv_gm1,
                       T theta, const double *w, hipStream_t s)
{
    int most = 0;
    for (int k = 0; k < nbox; ++k)
        for (int q = 0; q < ND; ++q) most = std::max(most, fs.b[k].n[(q + 1) % 3] * fs.b[k].n[(q + 2) % 3]);
    const dim3 grid((most + FB - 1) / FB, nbox * ND * 2);
    if (solver == SOLVER_HLL)
        hipLaunchKernelGGL((k_box_flux<ND, SOLVER_HLL, T>), grid, dim3(FB), 0, s, u, g, fs, gamma, gm1, inv_gm1, theta, w);
    else
        hipLaunchKernelGGL((k_box_flux<ND, SOLVER_HLLC, T>), grid, dim3(FB), 0, s, u, g, fs, gamma, gm1, inv_gm1, theta, w);
    return hipGetLastError();
}


// up to two clock updates in order (op < 0: none)
__global__ void __launch_bounds__(64) k_clock(FmrClock *c, int op0, int l0, int op1, int l1, int nlev,
                                               unsigned long long *rate_bits, double cfl, double dt_fixed)
{
    if (threadIdx.x != 0) return;
    clock_op(c, op0, l0, nlev, rate_bits, cfl, dt_fixed);
    clock_op(c, op1, l1, nlev, rate_bits, cfl, dt_fixed);
}

}  // namespace

hipError_t launch_clock(FmrClock *clock, int op0, int l0, int op1, int l1, int nlev, unsigned long long *rate_bits,
                        double cfl, double dt_fixed, hipStream_t s)
{
    hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, s, clock, op0, l0, op1, l1, nlev, rate_bits, cfl, dt_fixed);
    return hipGetLastError();
}

template <typename T>
RideJob<T> prolong_job(T *fine, T *fine2, const Grid &fg, const T *parent, const Grid &pg, const Box &parent_box,
                       int ndim, T gm1, const ClockOps &ck)
{
    RideJob<T> j{};
    j.fine = fine;
    j.fine2 = fine2;
    j.fg = fg;
    j.parent = parent;
    j.pg = pg;
    j.pb = parent_box;
    j.gm1 = gm1;
    j.inv_gm1 = T(1) / gm1;
    j.cells = fine == nullptr ? 0 : ndim == 1 ? shell_cells<1>(fg) : ndim == 2 ? shell_cells<2>(fg) : shell_cells<3>(fg);
    j.blocks = 0;
    j.ck = ck;
    return j;
}

template <typename T>
hipError_t launch_prolong(T *fine, T *fine2, const Grid &fg, const T *parent, const Grid &pg, const Box &parent_box,
                          int ndim, T gamma, T gm1, const ClockOps &ck, hipStream_t s)
{
    (void)gamma;
    RideJob<T> j = prolong_job<T>(fine, fine2, fg, parent, pg, parent_box, ndim, gm1, ck);
    j.blocks = std::max(1, (j.cells + SB - 1) / SB);
    const dim3 grid((unsigned)j.blocks);
    if (ndim == 1) hipLaunchKernelGGL((k_prolong<1, T>), grid, dim3(SB), 0, s, j);
    else if (ndim == 2) hipLaunchKernelGGL((k_prolong<2, T>), grid, dim3(SB), 0, s, j);
    else hipLaunchKernelGGL((k_prolong<3, T>), grid, dim3(SB), 0, s, j);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_box_flux(const T *u, const Grid &g, int nbox, const Box *boxes, double *const (*acc)[3][2],
                           const int *assign, int ndim, int solver, T gamma, T gm1, T inv_gm1, T theta,
                           const double *w, hipStream_t s)
{
    if (nbox < 1 || nbox > 2) return hipErrorInvalidValue;
    FluxSet fs{};
    for (int k = 0; k < nbox; ++k) {
        fs.b[k] = boxes[k];
        fs.assign[k] = assign[k];
        for (int q = 0; q < 3; ++q)
            for (int side = 0; side < 2; ++side) fs.acc[k][q][side] = acc[k][q][side];
    }
    if (ndim == 1) return box_flux_nd<1>(u, g, fs, nbox, solver, gamma, gm1, inv_gm1, theta, w, s);
    if (ndim == 2) return box_flux_nd<2>(u, g, fs, nbox, solver, gamma, gm1, inv_gm1, theta, w, s);
    return box_flux_nd<3>(u, g, fs, nbox, solver, gamma, gm1, inv_gm1, theta, w, s);
}

template <typename T>
hipError_t launch_reflux_restrict(T *u, const Grid &g, const Box &child_box, int ndim, const double *const coarse[3][2],
                                  const double *const fine[3][2], const double idq[3], const T *child, const Grid &cg,
                                  const RideJob<T> *ride, hipStream_t s)
{
    RefluxSet r{};
    int most = 0;
    for (int q = 0; q < 3; ++q) {
        for (int side = 0; side < 2; ++side) {
            r.c[q][side] = coarse[q][side];
            r.f[q][side] = fine[q][side];
        }
        r.idq[q] = idq[q];
        if (q < ndim) {
            const int r1 = q == 0 ? 1 : 0, r2 = q == 2 ? 1 : 2;
            most = std::max(most, child_box.n[r1] * child_box.n[r2]);
        }
    }
    const int rblocks = (most + FB - 1) / FB;
    const int64_t cells = (int64_t)child_box.n[0] * child_box.n[1] * child_box.n[2];
    const int64_t rcblocks = (int64_t)ndim * rblocks + (cells + FB - 1) / FB;
    RideJob<T> j{};
    if (ride) {
        j = *ride;
        j.blocks = (j.cells > 0 || j.ck.c) ? std::max(1, (j.cells + FB - 1) / FB) : 0;
    }
    const int64_t blocks = rcblocks + j.blocks;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    const int rc = (int)rcblocks;
    if (ndim == 1)
        hipLaunchKernelGGL((k_reflux_restrict<1, T>), grid, dim3(FB), 0, s, u, g, child_box, r, child, cg, rblocks, rc, j);
    else if (ndim == 2)
        hipLaunchKernelGGL((k_reflux_restrict<2, T>), grid, dim3(FB), 0, s, u, g, child_box, r, child, cg, rblocks, rc, j);
    else
        hipLaunchKernelGGL((k_reflux_restrict<3, T>), grid, dim3(FB), 0, s, u, g, child_box, r, child, cg, rblocks, rc, j);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_box_rate(const T *u, const Grid &g, const Box &box, int ndim, T gamma, T gm1, const double idq[3],
                           unsigned long long *rate_bits, hipStream_t s)
{
    const int64_t cells = (int64_t)box.n[0] * box.n[1] * box.n[2];
    const dim3 grid((unsigned)std::min<int64_t>((cells + TB - 1) / TB, 1024));
    if (ndim == 1)
        hipLaunchKernelGGL((k_box_rate<1, T>), grid, dim3(TB), 0, s, u, g, box, gamma, gm1, idq[0], idq[1], idq[2], rate_bits);
    else if (ndim == 2)
        hipLaunchKernelGGL((k_box_rate<2, T>), grid, dim3(TB), 0, s, u, g, box, gamma, gm1, idq[0], idq[1], idq[2], rate_bits);
    else
        hipLaunchKernelGGL((k_box_rate<3, T>), grid, dim3(TB), 0, s, u, g, box, gamma, gm1, idq[0], idq[1], idq[2], rate_bits);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_leaf_totals(const T *u, const Grid &g, const Box &box, const Box &hole, int ndim, double dv,
                              double *partials, hipStream_t s)
{
    const dim3 grid(box.n[1], box.n[2]);
    if (ndim == 1) hipLaunchKernelGGL((k_leaf_totals<1, T>), grid, dim3(TB), 0, s, u, g, box, hole, dv, partials);
    else if (ndim == 2) hipLaunchKernelGGL((k_leaf_totals<2, T>), grid, dim3(TB), 0, s, u, g, box, hole, dv, partials);
    else hipLaunchKernelGGL((k_leaf_totals<3, T>), grid, dim3(TB), 0, s, u, g, box, hole, dv, partials);
    return hipGetLastError();
}

#define HY_FMR_INST(T)                                                                                               \
    template hipError_t launch_prolong<T>(T *, T *, const Grid &, const T *, const Grid &, const Box &, int, T, T,   \
                                          const ClockOps &, hipStream_t);                                            \
    template hipError_t launch_box_flux<T>(const T *, const Grid &, int, const Box *, double *const(*)[3][2],        \
                                           const int *, int, int, T, T, T, T, const double *, hipStream_t);          \
    template hipError_t launch_reflux_restrict<T>(T *, const Grid &, const Box &, int, const double *const[3][2],    \
                                                  const double *const[3][2], const double[3], const T *,             \
                                                  const Grid &, const RideJob<T> *, hipStream_t);                    \
    template RideJob<T> prolong_job<T>(T *, T *, const Grid &, const T *, const Grid &, const Box &, int, T,          \
                                       const ClockOps &);                                                            \
    template hipError_t launch_box_rate<T>(const T *, const Grid &, const Box &, int, T, T, const double[3],         \
                                           unsigned long long *, hipStream_t);                                       \
    template hipError_t launch_leaf_totals<T>(const T *, const Grid &, const Box &, const Box &, int, double,        \
                                              double *, hipStream_t);
HY_FMR_INST(float)
HY_FMR_INST(double)
#undef HY_FMR_INST

}  // namespace hy
