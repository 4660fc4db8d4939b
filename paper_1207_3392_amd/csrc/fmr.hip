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

#include <algorithm>

namespace hy {
namespace {

constexpr int FB = 64;   // threads per block of the shell and face kernels
constexpr int TB = 256;  // threads per block of the reductions

constexpr int SB = 256;  // threads per block of the exterior-shell kernels

// The exterior cells of a padded array, enumerated flat: first the rows that
// lie wholly in the exterior (every x), then the NG cells at each x end of
// the remaining rows.
template <int ND>
__host__ __device__ inline int shell_full_rows(const Grid &g)
{
    if constexpr (ND == 1) return 0;
    if constexpr (ND == 2) return 2 * FMR_NG;
    return 2 * FMR_NG * g.m[1] + (g.m[2] - 2 * FMR_NG) * 2 * FMR_NG;
}

template <int ND>
__host__ __device__ inline int shell_cells(const Grid &g)
{
    int part = 1;
    if constexpr (ND >= 2) part *= g.m[1] - 2 * FMR_NG;
    if constexpr (ND >= 3) part *= g.m[2] - 2 * FMR_NG;
    return shell_full_rows<ND>(g) * g.m[0] + part * 2 * FMR_NG;
}

template <int ND>
__device__ __forceinline__ void shell_cell(const Grid &g, int s, int (&c)[3])
{
    const int full = shell_full_rows<ND>(g) * g.m[0];
    c[1] = 0;
    c[2] = 0;
    if (s < full) {
        const int r = s / g.m[0];
        c[0] = s - r * g.m[0];
        if constexpr (ND == 2) {
            c[1] = r < FMR_NG ? r : g.m[1] - 2 * FMR_NG + r;
        } else if constexpr (ND == 3) {
            const int slab = FMR_NG * g.m[1];  // rows of the low (or high) z exterior
            if (r < 2 * slab) {
                const int h = r / slab, rr = r - h * slab;
                c[2] = (h ? g.m[2] - FMR_NG : 0) + rr / g.m[1];
                c[1] = rr % g.m[1];
            } else {
                const int rr = r - 2 * slab, jj = rr % (2 * FMR_NG);
                c[2] = FMR_NG + rr / (2 * FMR_NG);
                c[1] = jj < FMR_NG ? jj : g.m[1] - 2 * FMR_NG + jj;
            }
        }
    } else {
        const int p = s - full, row = p / (2 * FMR_NG), x = p - row * 2 * FMR_NG;
        c[0] = x < FMR_NG ? x : g.m[0] - 2 * FMR_NG + x;
        if constexpr (ND == 2) c[1] = FMR_NG + row;
        if constexpr (ND == 3) {
            const int ny = g.m[1] - 2 * FMR_NG;
            c[2] = FMR_NG + row / ny;
            c[1] = FMR_NG + row % ny;
        }
    }
}

__device__ __forceinline__ void clock_op(FmrClock *c, int op, int l, int nlev, unsigned long long *rate_bits,
                                         double cfl, double dt_fixed)
{
    switch (op) {
    case CLOCK_RESET:
        for (int i = 0; i < nlev; ++i) c[i].t = 0.0;
        for (int k = 0; k < FMR_RATE_SLOTS; ++k) rate_bits[k] = 0ull;
        break;
    case CLOCK_DEEPEST:
    case CLOCK_DEEPEST_KEEP: {
        unsigned long long rb = 0ull;
        for (int k = 0; k < FMR_RATE_SLOTS; ++k) {
            rb = rb > rate_bits[k] ? rb : rate_bits[k];
            if (op == CLOCK_DEEPEST) rate_bits[k] = 0ull;
        }
        c[l].dt = dt_fixed > 0.0 ? dt_fixed : cfl / __longlong_as_double((long long)rb);
        break;
    }
    case CLOCK_COARSE: c[l].dt = c[l + 1].t - c[l].t; break;
    case CLOCK_PROVISIONAL: c[l].dtp = c[l + 1].t - c[l].t; break;
    case CLOCK_ADVANCE: c[l].t += c[l].dt; break;
    default: break;
    }
}

template <int ND, typename T>
__global__ void __launch_bounds__(SB) k_prolong(T *fine, T *fine2, Grid fg, const T *parent, Grid pg, Box pb, T gm1,
                                                 T inv_gm1, ClockOps ck)
{
    // clock updates that ride on this launch (none of its threads reads the
    // clocks; the kernels after it do)
    if (blockIdx.x == 0 && threadIdx.x == 0 && ck.c) {
        clock_op(ck.c, ck.op0, ck.l0, ck.nlev, ck.rate, ck.cfl, ck.dt_fixed);
        clock_op(ck.c, ck.op1, ck.l1, ck.nlev, ck.rate, ck.cfl, ck.dt_fixed);
    }
    const int sc = blockIdx.x * SB + threadIdx.x;
    if (sc < shell_cells<ND>(fg)) {
        int c3[3];
        shell_cell<ND>(fg, sc, c3);
        int p3[3], s3[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (q < ND) {
                const int r = c3[q] - FMR_NG;  // offset from the first interior cell
                p3[q] = pb.lo[q] + (r >> 1);   // floor(r / 2)
                s3[q] = r & 1;                 // 0: low child, 1: high child
            } else {
                p3[q] = 0;
                s3[q] = 0;
            }
        }
        T w0[ND + 2], wc[ND + 2];
        load_prim<ND>(parent, pg, at(pg, p3[0], p3[1], p3[2]), gm1, w0);
#pragma unroll
        for (int v = 0; v < ND + 2; ++v) wc[v] = w0[v];
#pragma unroll
        for (int q = 0; q < ND; ++q) {
            int lo3[3] = {p3[0], p3[1], p3[2]}, hi3[3] = {p3[0], p3[1], p3[2]};
            lo3[q] -= 1;
            hi3[q] += 1;
            T wm[ND + 2], wp[ND + 2];
            load_prim<ND>(parent, pg, at(pg, lo3[0], lo3[1], lo3[2]), gm1, wm);
            load_prim<ND>(parent, pg, at(pg, hi3[0], hi3[1], hi3[2]), gm1, wp);
            // minmod (theta = 1) as twice the slope; the child sits at +/- 1/4
            // of the parent width, so it moves by +/- slope2 / 8
            const T h = s3[q] ? T(0.125) : T(-0.125);
#pragma unroll
            for (int v = 0; v < ND + 2; ++v) wc[v] += h * slope2_mm(wm[v], w0[v], wp[v], T(2));
        }
        const int64_t c = at(fg, c3[0], c3[1], c3[2]);
        T uc[ND + 2], ke = T(0);
        uc[0] = wc[0];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            uc[1 + d] = wc[0] * wc[1 + d];
            ke += wc[1 + d] * wc[1 + d];
        }
        uc[ND + 1] = wc[ND + 1] * inv_gm1 + T(0.5) * wc[0] * ke;
#pragma unroll
        for (int v = 0; v < ND + 2; ++v) {
            fine[v * fg.vs + c] = uc[v];
            if (fine2) fine2[v * fg.vs + c] = uc[v];
        }
    }
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
                                                        int rblocks)
{
    const int bid = blockIdx.x;
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
hipError_t launch_prolong(T *fine, T *fine2, const Grid &fg, const T *parent, const Grid &pg, const Box &parent_box,
                          int ndim, T gamma, T gm1, const ClockOps &ck, hipStream_t s)
{
    (void)gamma;
    const T inv_gm1 = T(1) / gm1;
    const int cells = ndim == 1 ? shell_cells<1>(fg) : ndim == 2 ? shell_cells<2>(fg) : shell_cells<3>(fg);
    const dim3 grid((cells + SB - 1) / SB);
    if (ndim == 1) hipLaunchKernelGGL((k_prolong<1, T>), grid, dim3(SB), 0, s, fine, fine2, fg, parent, pg, parent_box, gm1,
                           inv_gm1, ck);
    else if (ndim == 2) hipLaunchKernelGGL((k_prolong<2, T>), grid, dim3(SB), 0, s, fine, fine2, fg, parent, pg, parent_box, gm1,
                           inv_gm1, ck);
    else hipLaunchKernelGGL((k_prolong<3, T>), grid, dim3(SB), 0, s, fine, fine2, fg, parent, pg, parent_box, gm1,
                           inv_gm1, ck);
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
                                  hipStream_t s)
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
    const int64_t blocks = (int64_t)ndim * rblocks + (cells + FB - 1) / FB;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    if (ndim == 1)
        hipLaunchKernelGGL((k_reflux_restrict<1, T>), grid, dim3(FB), 0, s, u, g, child_box, r, child, cg, rblocks);
    else if (ndim == 2)
        hipLaunchKernelGGL((k_reflux_restrict<2, T>), grid, dim3(FB), 0, s, u, g, child_box, r, child, cg, rblocks);
    else
        hipLaunchKernelGGL((k_reflux_restrict<3, T>), grid, dim3(FB), 0, s, u, g, child_box, r, child, cg, rblocks);
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
                                                  const Grid &, hipStream_t);                                        \
    template hipError_t launch_box_rate<T>(const T *, const Grid &, const Box &, int, T, T, const double[3],         \
                                           unsigned long long *, hipStream_t);                                       \
    template hipError_t launch_leaf_totals<T>(const T *, const Grid &, const Box &, const Box &, int, double,        \
                                              double *, hipStream_t);
HY_FMR_INST(float)
HY_FMR_INST(double)
#undef HY_FMR_INST

}  // namespace hy
