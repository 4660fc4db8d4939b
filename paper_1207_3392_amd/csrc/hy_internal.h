// Internal declarations shared by the library's HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hy {

constexpr int RATE_SLOTS = 32;

// Device control block: one per patch, inside the caller's workspace.
// rate[s][k] holds the bits of a positive double: the max over the cells of
// the blocks with id = k (mod RATE_SLOTS) of (|v_q| + c) / dq, for the state in
// parity slot s (the CFL rate is the max over k).  Positive doubles order like
// their bit patterns, so unsigned 64-bit atomic max reduces them; spreading
// blocks over slots keeps the atomics uncontended.
struct DevCtl {
    double time[2];
    unsigned long long rate[2][RATE_SLOTS];
    unsigned int err;
    unsigned int pad[3];
    double totals[8];
};

// LIM_THETA_PADDED: the generalised-minmod limiter on a view of a larger
// array (a refined level, or part of one): the cells updated are the n cells
// starting at storage cell voff of an array of extents vm, and the 2 cells
// around them on each side of every active dimension are read as they are
// (filled by the caller); no boundary kind applies.
enum { LIM_THETA = 0, LIM_LEARNED = 1, LIM_THETA_PADDED = 2 };
// Riemann solvers; the switch is HLLC with HLL at faces transverse to a shock
enum { SOLVER_HLL = 0, SOLVER_HLLC = 1, SOLVER_HLLC_SWITCH = 2 };
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2 };

// How a stage obtains dt: from the host argument, from the device control
// block (dt = min(cfl / rate, t_end - t)), or from a double in device memory
// (dt_dev; the multilevel driver keeps each level's step there).
enum { DT_HOST = 0, DT_DEVICE = 1, DT_PTR = 2 };

// A box of cells of an array: first cell (array coordinates) and cells per
// dimension (1 along unused dimensions).
struct Box {
    int lo[3];
    int n[3];
};

// Dense array extents and variable stride.
struct Grid {
    int m[3];
    int64_t vs;
};

// Face fluxes that a padded stage launch computes beside its cell update
// (nbox = 0: none): for each of nbox boxes of the stage input, the fluxes
// through its low and high faces along every active q from the input's
// generalised-minmod face states, acc[k][q][side][v * faces + t] += dt / 2 *
// F (= when assign[k] != 0), t over the box's cells transverse to q, the
// lower transverse dimension fastest.  The launcher adds blocks workgroups
// per (box, q, side) after the tile workgroups.
struct BoxFluxes {
    Box b[2];
    double *acc[2][3][2];
    int assign[2];
    int nbox;
    int blocks;
};

// A multilevel level's clock in device memory (its time, the step of its
// next full step and of its next provisional half-step) and clock updates
// carried by another launch (c == nullptr: none); see hy_fmr.h.
struct FmrClock {
    double t, dt, dtp, pad;
};
struct ClockOps {
    FmrClock *c;
    int op0, l0, op1, l1, nlev;
    unsigned long long *rate;
    double cfl, dt_fixed;
};

// Work that rides on another launch of the multilevel step: the prolongation
// of a padded level's exterior from its parent (cells > 0) and/or clock
// updates (ck.c), done by `blocks` extra workgroups appended to the host
// launch (the launcher sets blocks for its workgroup size).  The host launch
// must neither read nor write what the job touches; see hy_fmr.h.
template <typename T>
struct RideJob {
    T *fine, *fine2;
    Grid fg;
    const T *parent;
    Grid pg;
    Box pb;
    T gm1, inv_gm1;
    int cells, blocks;
    ClockOps ck;
};

template <typename T>
struct StageArgs {
    const T *uin;     // state read with the stencil (U^n in stage 1, U^(1) in stage 2)
    T *uout;          // output (U^(1) in stage 1; U^{n+1} over U^n in stage 2)
    const T *u0;      // stage 2: U^n, read only at the thread's own cell (aliases uout)
    const float *slopes;  // learned limiter: (ndim * nv, ncell) slopes of the stage input
    int64_t n[3];
    int64_t vstride;  // elements between variables
    T idx[3];         // 1 / dq
    T gamma, gm1, inv_gm1, theta;
    T accel[3];
    int bc[3][2];
    int zchunk;       // planes per block along z (3D)
    int tiles_x, tiles_y, ntiles;  // tile grid (set by the launcher)
    DevCtl *ctl;
    int parity;       // slot of the input state's time / rate
    int dt_mode;
    double dt_host, cfl, t_end;
    const double *dt_dev;  // DT_PTR: the step
    int voff[3], vm[3];    // LIM_THETA_PADDED: first updated cell and extents of the storage
    BoxFluxes bf;          // LIM_THETA_PADDED: face fluxes of the input computed in the same launch
    int nbfwg;             // LIM_THETA_PADDED: workgroups of bf (set by the launcher)
    RideJob<T> ride;       // LIM_THETA_PADDED: a job riding on the launch (after bf's workgroups)
};

struct LaunchCfg {
    int bx;       // plane tile width (block = bx x by threads)
    int by;       // plane tile rows
    int zchunk;   // planes per block along z
};

// Stage launchers (defined in stage.hip).  Return hipSuccess or the launch error.
template <typename T>
hipError_t launch_stage(int ndim, int solver, int stage, int limiter, const LaunchCfg &cfg,
                        const StageArgs<T> &a, hipStream_t s);

// Threshold of the HLLC switch's shock detector (relative pressure jump
// across a cell; the stage kernel evaluates the detector).
constexpr double SHOCK_EPS = 0.5;

// Device-side helpers (defined in reduce.hip).
template <typename T>
hipError_t launch_prim_to_cons(T *u, int64_t ncell, int64_t vstride, int ndim, T gm1, T inv_gm1,
                               hipStream_t s);
template <typename T>
hipError_t launch_cons_to_prim(const T *u, T *w, int64_t ncell, int64_t vstride, int ndim, T gm1,
                               hipStream_t s);
template <typename T>
hipError_t launch_cfl_rate(const T *u, int64_t n0, int64_t n1, int64_t n2, int64_t vstride, int ndim,
                           T gamma, T gm1, const double *idx, DevCtl *ctl, int slot, hipStream_t s);
template <typename T>
hipError_t launch_totals(const T *u, int64_t ncell, int64_t vstride, int ndim, double dv,
                         double *partials, int nblocks, DevCtl *ctl, hipStream_t s);

hipError_t launch_ctl_reset_rate(DevCtl *ctl, int slot, hipStream_t s);
hipError_t launch_ctl_init(DevCtl *ctl, hipStream_t s);

constexpr int TOTALS_BLOCKS = 512;

}  // namespace hy
