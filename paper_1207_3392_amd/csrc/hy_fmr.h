// Fixed multilevel refinement: device kernels' launchers (internal).
//
// Levels are nested boxes refined by two along every active dimension.  A
// refined level lives in a padded array: its n cells per active dimension
// plus NG = 2 exterior cells on each side, which hold values prolonged from
// the next coarser level; the stage kernels (padded mode) update the interior
// and read the exterior as the stencil's ghost cells.  All arrays are SoA (variable stride vs), x fastest;
// "box" arguments are cell ranges in the coordinates of the array they index.
#pragma once

#include "hy_internal.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hy {

constexpr int FMR_NG = 2;

// A level's clock (FmrClock, hy_internal.h) lives in device memory: its
// time, the step of its next full step and of its next provisional
// half-step.  Kernels read their steps from there, so a global step needs no
// host round trip.

enum {
    CLOCK_RESET = 0,
    CLOCK_DEEPEST = 1,
    CLOCK_COARSE = 2,
    CLOCK_PROVISIONAL = 3,
    CLOCK_ADVANCE = 4,
    CLOCK_DEEPEST_KEEP = 5
};

// The CFL rate is reduced into FMR_RATE_SLOTS words (workgroup b into word
// b mod FMR_RATE_SLOTS), so the atomics of a reduction never queue on one
// address; readers take the max over the words.
constexpr int FMR_RATE_SLOTS = 32;

// One launch applies the clock updates op0 (on level l0), then op1 (on l1),
// on a single thread; an op < 0 is skipped.  The updates:
//  RESET        every level's time to 0 and the rate words to 0;
//  DEEPEST      dt of level l = dt_fixed if > 0, else cfl / (the max of the
//               rate words), which are then cleared;
//  DEEPEST_KEEP the same from rate words that belong to someone else (a
//               patch's control block), left as they are;
//  COARSE       dt of level l = t(l + 1) - t(l) (the child's two steps);
//  PROVISIONAL  dtp of level l = t(l + 1) - t(l) (the child's first step);
//  ADVANCE      t(l) += dt(l).
hipError_t launch_clock(FmrClock *clock, int op0, int l0, int op1, int l1, int nlev, unsigned long long *rate_bits,
                        double cfl, double dt_fixed, hipStream_t s);

// Clock updates carried by another launch: ClockOps (hy_internal.h).

// Exterior of the padded level (fine) from its parent: each exterior cell at
// fine offset r from the level's first interior cell takes its parent
// cell's primitives plus +/- 1/4 of the parent's minmod-limited differences
// along each active dimension, stored as conserved variables into fine and,
// when not null, fine2 (the level's stage state).  parent_box names the
// parent cells the level refines.  The clock updates ck (if any) run in the
// same launch.
template <typename T>
hipError_t launch_prolong(T *fine, T *fine2, const Grid &fg, const T *parent, const Grid &pg, const Box &parent_box,
                          int ndim, T gamma, T gm1, const ClockOps &ck, hipStream_t s);

// Fluxes through the low and high faces of each of nbox (1 or 2) boxes of
// the array u along every active q (the unpadded coarsest level; a padded
// level's stage launch computes the same fluxes in workgroups of its own), from its generalised-minmod face states
// (a box needs two cells of u beyond each face), in one launch:
// acc[k][q][side][v * faces + t] += w * F for box k (= w * F when
// assign[k] != 0), w = *dt / 2 (a stage's share of the step), t running
// over the box's cells transverse to q, the lower transverse dimension
// fastest (x for faces normal to y or z, so neighbouring threads read
// neighbouring cells).
template <typename T>
hipError_t launch_box_flux(const T *u, const Grid &g, int nbox, const Box *boxes, double *const (*acc)[3][2],
                           const int *assign, int ndim, int solver, T gamma, T gm1, T inv_gm1, T theta,
                           const double *dt, hipStream_t s);

// After the child's two steps, in one launch: the coarse/fine replacement
// (every parent cell just outside child_box takes (fine - coarse) / dq of
// the flux through its face into the box, sign by side, the fine value being
// the mean over the 2^(d-1) child faces of the child's accumulated boundary
// fluxes, layout of launch_box_flux over the child's interior) and the
// restriction (every parent cell of child_box becomes the mean of its 2^d
// children, the child being a padded level, interior at offset NG).  The two
// touch disjoint parent cells.
// A job riding on the launch (ride != nullptr: RideJob, hy_internal.h) runs
// in extra workgroups after these.
template <typename T>
hipError_t launch_reflux_restrict(T *u, const Grid &g, const Box &child_box, int ndim, const double *const coarse[3][2],
                                  const double *const fine[3][2], const double idq[3], const T *child, const Grid &cg,
                                  const RideJob<T> *ride, hipStream_t s);

// The RideJob that launch_prolong's arguments describe (cells set, blocks
// left for the host launch's launcher).
template <typename T>
RideJob<T> prolong_job(T *fine, T *fine2, const Grid &fg, const T *parent, const Grid &pg, const Box &parent_box,
                       int ndim, T gm1, const ClockOps &ck);

// max over the cells of box of (|v_q| + c_s) / dq into the FMR_RATE_SLOTS
// words rate_bits (the bits of a positive double; unsigned atomic max).
template <typename T>
hipError_t launch_box_rate(const T *u, const Grid &g, const Box &box, int ndim, T gamma, T gm1, const double idq[3],
                           unsigned long long *rate_bits, hipStream_t s);

// Per row (j, k) of box, dv times the sums of D, S_q and G over the row's
// cells outside hole (hole.n[0] == 0: no hole) into partials[row * 5 + slot]
// (slots D, S_x, S_y, S_z, G).
template <typename T>
hipError_t launch_leaf_totals(const T *u, const Grid &g, const Box &box, const Box &hole, int ndim, double dv,
                              double *partials, hipStream_t s);

}  // namespace hy
