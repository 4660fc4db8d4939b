// Device helpers of the multilevel step shared by the multilevel kernels
// and the stage kernel's padded launches (internal): the enumeration of a
// padded level's exterior shell, the clock updates, and the prolongation of
// the exterior from the parent (Sec. 2), which a launch of its own or extra
// workgroups of another launch (RideJob) carry out.
#pragma once

#include "hy_fmr.h"
#include "hy_face.h"

namespace hy {
namespace {

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

// One exterior cell (shell index sc) of the job's level: the parent cell's
// primitives plus +/- 1/4 of the parent's minmod-limited differences along
// each active dimension, stored as conserved variables into fine and, when
// not null, fine2 (the level's stage state).
template <int ND, typename T>
__device__ __forceinline__ void prolong_cell(const RideJob<T> &j, int sc)
{
    int c3[3];
    shell_cell<ND>(j.fg, sc, c3);
    int p3[3], s3[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (q < ND) {
            const int r = c3[q] - FMR_NG;  // offset from the first interior cell
            p3[q] = j.pb.lo[q] + (r >> 1);  // floor(r / 2)
            s3[q] = r & 1;                  // 0: low child, 1: high child
        } else {
            p3[q] = 0;
            s3[q] = 0;
        }
    }
    T w0[ND + 2], wc[ND + 2];
    load_prim<ND>(j.parent, j.pg, at(j.pg, p3[0], p3[1], p3[2]), j.gm1, w0);
#pragma unroll
    for (int v = 0; v < ND + 2; ++v) wc[v] = w0[v];
#pragma unroll
    for (int q = 0; q < ND; ++q) {
        int lo3[3] = {p3[0], p3[1], p3[2]}, hi3[3] = {p3[0], p3[1], p3[2]};
        lo3[q] -= 1;
        hi3[q] += 1;
        T wm[ND + 2], wp[ND + 2];
        load_prim<ND>(j.parent, j.pg, at(j.pg, lo3[0], lo3[1], lo3[2]), j.gm1, wm);
        load_prim<ND>(j.parent, j.pg, at(j.pg, hi3[0], hi3[1], hi3[2]), j.gm1, wp);
        // minmod (theta = 1) as twice the slope; the child sits at +/- 1/4
        // of the parent width, so it moves by +/- slope2 / 8
        const T h = s3[q] ? T(0.125) : T(-0.125);
#pragma unroll
        for (int v = 0; v < ND + 2; ++v) wc[v] += h * slope2_mm(wm[v], w0[v], wp[v], T(2));
    }
    const int64_t c = at(j.fg, c3[0], c3[1], c3[2]);
    T uc[ND + 2], ke = T(0);
    uc[0] = wc[0];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        uc[1 + d] = wc[0] * wc[1 + d];
        ke += wc[1 + d] * wc[1 + d];
    }
    uc[ND + 1] = wc[ND + 1] * j.inv_gm1 + T(0.5) * wc[0] * ke;
#pragma unroll
    for (int v = 0; v < ND + 2; ++v) {
        j.fine[v * j.fg.vs + c] = uc[v];
        if (j.fine2) j.fine2[v * j.fg.vs + c] = uc[v];
    }
}

// Workgroup wg (of j.blocks, nthreads threads each) of a riding job: the
// clock updates on its first thread, then its share of the shell cells.
template <int ND, typename T>
__device__ __forceinline__ void ride_run(const RideJob<T> &j, int wg, int tid, int nthreads)
{
    if (wg == 0 && tid == 0 && j.ck.c) {
        clock_op(j.ck.c, j.ck.op0, j.ck.l0, j.ck.nlev, j.ck.rate, j.ck.cfl, j.ck.dt_fixed);
        clock_op(j.ck.c, j.ck.op1, j.ck.l1, j.ck.nlev, j.ck.rate, j.ck.cfl, j.ck.dt_fixed);
    }
    for (int sc = wg * nthreads + tid; sc < j.cells; sc += j.blocks * nthreads) prolong_cell<ND>(j, sc);
}

}  // namespace
}  // namespace hy
