/*
 * hydro.h -- C ABI of the gfx950 finite-volume hydrodynamics library
 * (libhydro.so).  It advances the nonrelativistic Euler equations of
 * Cardall et al., "GenASiS I" (arXiv:1207.3392), Sec. 3, on one uniform
 * Cartesian patch held in GPU memory.
 *
 * Conventions shared by every entry point
 *  - Every function returns hy_status (0 = HY_OK, negative = error) and never
 *    throws; hy_last_error() gives a thread-local message for the last error.
 *  - Host arrays are structure-of-arrays (nv, nz, ny, nx), x fastest, over
 *    interior cells only, FP64.  nv = ndim + 2.  Conserved order (Sec. 3.5):
 *    D, S_1..S_ndim, G.  Primitive order: rho, v_1..v_ndim, p.  The baryon
 *    mass m is 1, so rho = D.  Unused dimensions have n = 1.
 *  - Device memory is owned by the caller: the library carves everything it
 *    needs out of one workspace the caller allocates (any device allocator,
 *    e.g. a torch uint8 tensor) after asking for its size.  The library itself
 *    allocates only its host-side handle.  hy_destroy frees the handle, never
 *    the workspace.
 *  - Work is enqueued on the caller's HIP stream (passed as void*, NULL =
 *    the default stream) without host synchronisation, except in the calls
 *    marked "synchronising".
 *  - A NaN, rho <= 0 or p <= 0 met by a kernel is latched in device memory and
 *    returned as HY_ESTATE by the next synchronising call; hy_set_state
 *    clears the latch.
 *  - One handle is not thread-safe; distinct handles are independent.
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HY_OK = 0,
    HY_EINVAL = -1,       /* bad argument (checked on the host before any launch) */
    HY_ENOMEM = -2,       /* workspace smaller than hy_*_workspace_bytes */
    HY_EDEVICE = -3,      /* a HIP runtime call failed */
    HY_ESTATE = -4,       /* NaN or rho <= 0 or p <= 0 latched on the device */
    HY_EUNSUPPORTED = -5  /* valid but not built (e.g. learned limiter in FP64) */
} hy_status;

typedef enum { HY_BC_PERIODIC = 0, HY_BC_OUTFLOW = 1, HY_BC_REFLECT = 2 } hy_bc;
/* HY_HLLC_SWITCH: HLLC, with HLL at the faces next to a shock that are
 * transverse to its direction of motion (Sec. 3.2, against odd-even
 * decoupling; the paper names no detector).  Detector: a cell is in a shock
 * moving along q when the pressures of its two neighbours along q differ by
 * more than 0.5 of the smaller one and the velocity along q decreases across
 * it; a face normal to r takes HLL when either adjacent cell is flagged
 * along some q != r.  The flags are recomputed from each stage's input (one
 * extra pass, one byte per cell in the workspace).  In 1D (and for batched
 * tubes) it is HLLC. */
typedef enum { HY_HLL = 0, HY_HLLC = 1, HY_HLLC_SWITCH = 2 } hy_solver;
typedef enum { HY_LIM_THETA = 0, HY_LIM_LEARNED = 1 } hy_limiter;
typedef enum { HY_PRIMITIVE = 0, HY_CONSERVED = 1 } hy_kind;

/*
 * Patch description.
 *  ndim        1, 2 or 3; n[q] >= 2 cells on active dimensions, 1 elsewhere;
 *              n[0] <= 2^20, n[1] and n[2] <= 65535, and one variable's array
 *              below 4 GiB (HY_EINVAL otherwise).
 *  lo, hi      box corners; cell width (hi - lo) / n (uniform grid, Sec. 3).
 *  gamma       ideal-gas index, p = (gamma - 1) e (Sec. 3.5, polytropic closure).
 *  bc[q][s]    boundary kind on the low (s = 0) / high (s = 1) face of
 *              dimension q.  Ghost cells are filled from cell-centre
 *              primitives: periodic wraps, outflow copies the nearest interior
 *              cell, reflecting mirrors and negates the normal velocity (the
 *              boundary step of Alg. 1 applied through ghost cells).  Periodic
 *              must be set on both faces of a dimension.
 *  precision   32 (FP32 state and fluxes; reductions in FP64) or 64.
 *  limiter     HY_LIM_THETA: generalised minmod of eq. MinMod with parameter
 *              theta in [1, 2] (1 = minmod, 2 = monotonized central).
 *              HY_LIM_LEARNED: the MLP slope limiter (weights via hy_set_mlp),
 *              FP32 only.
 *  accel       uniform acceleration a = -grad(Phi); the source is
 *              (0, rho a, rho v . a) (the external force and power of the
 *              Rayleigh-Taylor setup, Sec. 4.3.2).  Zeros: no source.
 */
typedef struct {
    int ndim;
    int64_t n[3];
    double lo[3];
    double hi[3];
    double gamma;
    int bc[3][2];
    int precision;
    int limiter;
    double theta;
    double accel[3];
} hy_patch_desc;

typedef struct hy_patch hy_patch; /* opaque, owned by the library */

/* Bytes of device workspace hy_init_patch needs for this description
 * (two state arrays plus small control blocks).  HY_EINVAL on a bad desc. */
hy_status hy_patch_workspace_bytes(const hy_patch_desc *desc, size_t *bytes);

/* Bind a patch to caller-owned device memory (at least the size above, any
 * alignment; contents need not be initialised) and a HIP stream.  The state is
 * undefined until hy_set_state.  *out receives the handle. */
hy_status hy_init_patch(const hy_patch_desc *desc, void *dev_workspace, size_t bytes,
                        void *hip_stream, hy_patch **out);

/* Copy a host FP64 state in (converted to the patch precision on the host,
 * primitives converted to conserved variables on the device), compute the
 * CFL rate of the new state, reset the simulation time to 0 and clear the
 * error latch.  Synchronising. */
hy_status hy_set_state(hy_patch *p, int kind, const double *host_soa);

/* Copy the current state out as FP64, conserved or primitive.  Synchronising;
 * HY_ESTATE if the latch is set (the array is still written). */
hy_status hy_get_state(hy_patch *p, int kind, double *host_soa_out);

/* One full two-stage Runge-Kutta step (eqs. Update, RungeKutta1-3) of size dt
 * with the HLL (eq. FluxHLL) or HLLC (eq. FluxHLLC) flux, or the switch.  dt must be finite
 * and > 0 (HY_EINVAL otherwise).  Asynchronous.  The second stage also
 * computes the CFL rate of the new state, so a following hy_cfl_dt launches
 * nothing. */
hy_status hy_step(hy_patch *p, double dt, int solver);

/* dt = cfl * min over cells and dimensions of dq / max(|v_q - c|, |v_q + c|)
 * (eq. courantTimeStep) for the current state.  Synchronising. */
hy_status hy_cfl_dt(hy_patch *p, double cfl, double *dt_out);

/* nsteps steps with the time step chosen on the device before each step:
 * dt = min(cfl * dt_CFL, t_end - t), t advanced on the device (the
 * single-level form of Alg. 2 without a host round trip).  Once t reaches
 * t_end the remaining steps leave the state unchanged.  Asynchronous. */
hy_status hy_advance(hy_patch *p, int nsteps, double cfl, double t_end, int solver);

/* The same nsteps device-dt steps as hy_advance, enqueued on the patch
 * stream as one HIP graph launch (the stage launches of every step only: no
 * memset, no event, no host wait).  The graph is captured on a private
 * stream of the library, instantiated, and kept per starting parity of the
 * patch's two state buffers; it is captured again when nsteps, cfl, t_end,
 * solver or the launch shape differ from the kept one.
 * hy_advance_graph_prepare does the capture alone (nothing runs, the state
 * is untouched), so a caller can keep it out of a timed region.  The
 * per-kernel timing of hy_set_timing covers launches outside graphs only
 * (a caller times a replay with its own events around it).  Refined
 * multilevel levels are rejected (HY_EUNSUPPORTED).  Results equal
 * hy_advance's bit for bit.  Asynchronous (apart from the capture). */
hy_status hy_advance_graph_prepare(hy_patch *p, int nsteps, double cfl, double t_end, int solver);
hy_status hy_advance_graph(hy_patch *p, int nsteps, double cfl, double t_end, int solver);

/* Simulation time accumulated by hy_step / hy_advance since hy_set_state.
 * Synchronising. */
hy_status hy_get_time(hy_patch *p, double *t_out);

/* FP64 totals sum_cells U_k dV in a fixed-order tree (bitwise reproducible),
 * out = (D, S_x, S_y, S_z, G), zeros for absent momentum components.
 * Synchronising. */
hy_status hy_conserved_totals(hy_patch *p, double out[5]);

/* Kinetic energy per component, out[q] = integral of rho v_q^2 / 2 over the
 * patch (the y component is the E_kin,y of the Kelvin-Helmholtz analysis,
 * Sec. 4.3.1), as dV times an FP64 fixed-order sum of S_q^2 / (2 D) over the
 * cells (bitwise reproducible); zeros for absent components.  Synchronising. */
hy_status hy_kinetic_energy(hy_patch *p, double out[3]);

/* Kinetic-energy spectrum of the Kelvin-Helmholtz analysis (Sec. 4.3.1) of
 * the patch's current state U^n, on the device: e[s], s = 0 .. nshell - 1,
 * is the energy density on the shell of wavenumbers |k| = 2 pi s / L (width
 * dk = 2 pi / L, s the integer nearest to the length of the integer
 * wavevector), from the discrete Fourier coefficients (divided by the cell
 * count) of the components of sqrt(rho) v with the box taken as periodic,
 * normalised so that sum_s e[s] dk is the integral of rho |v|^2 / 2 over the
 * box.  A 2D patch of N x N cells, N a power of two from 2 to 8192, on a
 * square box of side L (else HY_EUNSUPPORTED); nshell = floor(sqrt(2) N / 2
 * + 1/2) + 1.  The transform is FP64 and the shell sums are 64-bit
 * fixed-point at a scale of 2^-61 of the total (bitwise reproducible; each
 * term is truncated by less than 2^-61 of the total).
 * hy_spectrum_workspace_bytes gives the device workspace the call needs
 * (32 N^2 bytes plus a little; the caller owns it, nothing is kept); e is
 * host memory of cap >= nshell doubles (else HY_EINVAL, with *nshell set);
 * HY_ESTATE when a density is not positive.  Synchronising. */
hy_status hy_spectrum_workspace_bytes(hy_patch *p, size_t *bytes);
hy_status hy_kinetic_spectrum(hy_patch *p, void *dev_workspace, size_t bytes, double *e, int cap, int *nshell);

/* Learned limiter weights: n = 1249 FP32 values, W1[32][4], b1[32],
 * W2[32][32], b2[32], w3[32], b3.  Copied to the device (W1, W2 and w3 in
 * bfloat16, biases in FP32).  Required before stepping with HY_LIM_LEARNED.  Synchronising. */
hy_status hy_set_mlp(hy_patch *p, const float *weights, size_t n);

/* Per-kernel timing with HIP events on the patch stream (off by default).
 * While on, each stage launch is bracketed by events; hy_kernel_times
 * synchronises and returns the summed milliseconds and launch counts of the
 * first and second stage kernels since the last reset, then resets them. */
hy_status hy_set_timing(hy_patch *p, int on);
hy_status hy_kernel_times(hy_patch *p, double ms[2], int64_t launches[2]);

/* Name of the stage kernel configuration in use (for profiles). */
hy_status hy_kernel_config(hy_patch *p, char *buf, size_t len);

/* Launch shape of the stage kernels: a workgroup of bx x by threads owns a
 * bx x by tile of the x-y plane and marches along z over zchunk planes (3D;
 * zchunk = 1 otherwise).  The launch shape changes no result: every shape
 * computes the same cells with the same arithmetic.  Supported tiles:
 * 64x8, 64x4, 32x8 and (FP32) 32x16 in 2D and 3D, 64x1 in 1D; a patch starts
 * with a shape picked from its size (64x8, at least ~512 workgroups, at most
 * 64 planes per chunk).  The HLLC -> HLL switch keeps a shape of its own
 * (3D FP32: 32x8, at least ~1536 workgroups; else the same): hy_get_launch_cfg
 * reports the HLL/HLLC shape, hy_set_launch_cfg sets the shape of every
 * solver, hy_autotune the shape of the solver it tunes. */
typedef struct {
    int bx, by, zchunk;
} hy_launch_cfg;
hy_status hy_get_launch_cfg(hy_patch *p, hy_launch_cfg *out);
/* HY_EINVAL for an unsupported tile or a chunk outside 1..n_z (1 below 3D). */
hy_status hy_set_launch_cfg(hy_patch *p, const hy_launch_cfg *cfg);
/* Autotuner: times every supported tile (and in 3D the z chunks 8, 16, 32,
 * 64, 128 that fit, plus the starting one) over reps trials of both
 * Runge-Kutta stage kernels on the patch's current state with dt = 0 (each
 * stage reading U^n and writing the scratch stage state), on the patch
 * stream with HIP events (after a few settling trials of the starting
 * shape; two passes, each candidate's faster one counting), and keeps the
 * fastest shape unless the starting one is within 2 %; best and best_ms
 * (mean milliseconds per trial) may be NULL.  U^n, the time and the CFL
 * rate of U^n are unchanged; the scratch stage state is overwritten.  A
 * learned-limiter patch needs its weights (its slopes kernel has a fixed
 * shape and is not part of the trial).  Different z chunks may round
 * differently in the last place (the z faces at chunk starts are formed by
 * the chunk's entry code); tiles never change a result.  Synchronising. */
hy_status hy_autotune(hy_patch *p, int solver, int reps, hy_launch_cfg *best, double *best_ms);

hy_status hy_destroy(hy_patch *p);

const char *hy_last_error(void);

/* ---------------------------------------------------------------------
 * Batched tubes: many independent 1D patches of uneven length advanced to
 * one end time in a single persistent launch (captured once in a hipGraph
 * and replayed).  Each tube runs the single-level loop of Alg. 2 with its
 * own CFL time step, dt = min(cfl * dt_CFL, t_end - t), and the same
 * two-stage update as hy_step.  Every description must be ndim = 1,
 * precision = 32, limiter = HY_LIM_THETA, accel = 0 and n <= 6144
 * (HY_EUNSUPPORTED / HY_EINVAL otherwise).  Tube states are concatenated in
 * the caller's workspace; a workgroup holds one tube in LDS at a time, taking
 * tubes from a device queue in descending order of n^2 max(|v| + c) / L
 * (estimated from the states given to hy_batch_set_state). */
typedef struct hy_batch hy_batch;

hy_status hy_batch_workspace_bytes(const hy_patch_desc *descs, int count, size_t *bytes);
hy_status hy_batch_init(const hy_patch_desc *descs, int count, void *dev_workspace, size_t bytes,
                        void *hip_stream, hy_batch **out);
/* State of tube i (3 x n FP64, SoA); synchronising. */
hy_status hy_batch_set_state(hy_batch *b, int i, int kind, const double *host_soa);
/* Advance every tube from t = 0 to t_end; asynchronous (one graph launch). */
hy_status hy_batch_run_to(hy_batch *b, double t_end, double cfl, int solver);
/* Workgroup size of the batched kernel: 256, 512 or 1024 threads (a tube's
 * cells are dealt round-robin, 24, 12 or 6 register slots per thread); the
 * default is 1024.  The size changes no result.  HY_EINVAL otherwise. */
hy_status hy_batch_set_block(hy_batch *b, int threads);
hy_status hy_batch_get_block(hy_batch *b, int *threads);
/* Autotuner: runs the whole batch from its current state to t_end with each
 * workgroup size (the queue order and every tube's dt loop as in
 * hy_batch_run_to), times each launch with HIP events, keeps the fastest
 * (the current size unless another is at least 2 % faster) and restores
 * the state and the per-tube status as they were before; best
 * and best_ms may be NULL.  Synchronising. */
hy_status hy_batch_autotune(hy_batch *b, double t_end, double cfl, int solver, int *best_threads, double *best_ms);
/* Milliseconds of the last hy_batch_run_to launch (HIP events); synchronising. */
hy_status hy_batch_last_ms(hy_batch *b, double *ms);
/* State of tube i; synchronising; HY_ESTATE if that tube met a bad state. */
hy_status hy_batch_get_state(hy_batch *b, int i, int kind, double *host_soa_out);
/* Steps taken and time reached by tube i in the last run (0 steps at t = 0
 * before the first run); synchronising. */
hy_status hy_batch_status(hy_batch *b, int i, int64_t *steps, double *t);
hy_status hy_batch_destroy(hy_batch *b);

/* ---------------------------------------------------------------------
 * Learned slope limiter: training data and training on the device.  The
 * network (4 -> 32 -> 32 -> 1, ReLU) replaces eq. MinMod; its inputs are the
 * four one-sided differences of a 5-cell stencil of one primitive along one
 * dimension divided by s = max|d| + 1e-12 (|w_c| + 1e-30), and its output
 * times s is clamped to the TVD region 0 <= sign(D) sigma <= 2 min(|D-|,|D+|).
 *
 * Samples come from a fine FP32 patch of the plain method (periodic, every
 * active n divisible by 4, n >= 20): the state is restricted (averaged) onto
 * a 4x coarser grid; each (coarse cell, variable, dimension) is one sample
 * with inputs from the coarse 5-cell stencil and target the clamped
 * least-squares slope of the four fine sub-cell averages, 0.4 (-3 w1 - w2 +
 * w3 + 3 w4), divided by s.  x_dev receives (nsamples, 4) FP32, t_dev
 * (nsamples) FP32, both caller-allocated device buffers; sample index =
 * (q * nv + v) * ncoarse + coarse cell.  Asynchronous on the patch stream. */
hy_status hy_lim_sample_count(const hy_patch *fine, int64_t *nsamples);
hy_status hy_lim_samples_scratch_bytes(const hy_patch *fine, size_t *bytes);
hy_status hy_lim_make_samples(hy_patch *fine, void *dev_scratch, size_t scratch_bytes, float *x_dev, float *t_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * samples as hy_lim_make_samples, bit for bit, with the staging (coarse
 * primitives and sub-cell averages) in a library-owned static device array
 * of 64 MiB per GPU, held until the process ends, instead of a caller
 * scratch.  The caller passes the patch and the outputs x_dev, t_dev as
 * above.  HY_ENOMEM (nothing launched) when hy_lim_samples_scratch_bytes
 * exceeds 64 MiB.  Allocates nothing; the first call on a GPU looks up the
 * array's address there.  Every call on one GPU shares its array, which
 * keeps the last call's contents (each call writes all it reads, so nothing
 * needs clearing): calls that overlap on one GPU (other streams or threads)
 * race and must be serialised by the caller.  Asynchronous. */
hy_status hy_lim_make_samples_noalloc(hy_patch *fine, float *x_dev, float *t_dev);

/* Learned slopes of the current state of a HY_LIM_LEARNED patch (weights
 * set): out_dev (caller device buffer of ndim * nv * ncell FP32) receives
 * sigma[(q * nv + v) * ncell + cell], the per-cell difference slope of
 * primitive v along q after the TVD clamp.  Asynchronous. */
hy_status hy_lim_slopes(hy_patch *p, float *out_dev);

/* Trainer: FP32 master weights and Adam moments (beta1 0.9, beta2 0.999,
 * eps 1e-8) in a caller workspace.  One step evaluates the network forward
 * and backward on the samples idx_dev[0..batch) (bf16 MFMA operands, FP32
 * accumulation), reduces the gradient of the mean squared error of the raw
 * output against the target in a fixed order, and applies Adam with rate lr.
 * hy_trainer_gradient computes the same gradient without updating
 * (synchronising); hy_mlp_eval runs the limiter's inference kernel with the
 * trainer's current weights on x_dev (batch, 4) into y_dev (batch).
 * Inputs and targets must be finite: the matrix kernels evaluate 64 samples
 * together, and a non-finite input can turn the outputs (or the gradient) of
 * other samples of its group into NaN.  The sample generator and the learned
 * slopes never produce one from a finite state. */
typedef struct hy_trainer hy_trainer;
hy_status hy_trainer_workspace_bytes(size_t *bytes);
hy_status hy_trainer_init(void *dev_workspace, size_t bytes, const float *init_params, void *hip_stream,
                          hy_trainer **out);
hy_status hy_trainer_step(hy_trainer *tr, const float *x_dev, const float *t_dev, const int32_t *idx_dev,
                          int64_t batch, float lr);
hy_status hy_trainer_gradient(hy_trainer *tr, const float *x_dev, const float *t_dev, const int32_t *idx_dev,
                              int64_t batch, float *grad_host, float *loss_host);
hy_status hy_trainer_loss(hy_trainer *tr, float *loss_host);
hy_status hy_trainer_get_params(hy_trainer *tr, float *params_host);
hy_status hy_mlp_eval(hy_trainer *tr, const float *x_dev, float *y_dev, int64_t batch);
hy_status hy_trainer_destroy(hy_trainer *tr);

/* ---------------------------------------------------------------------
 * Fixed multilevel refinement (Sec. 2, the refinable mesh with its
 * prolongation and restriction; Sec. 3.6, Algs. Evolve, EvolveLevel and
 * StepLevel).  Level 0 is `base` (the whole box, its boundary kinds,
 * precision, gamma, theta; limiter must be HY_LIM_THETA, and the solver of
 * hy_fmr_step HY_HLL or HY_HLLC).  Level l >= 1 refines by two along every
 * active dimension the cells box_lo[l] .. box_lo[l] + box_n[l] - 1 of level
 * l - 1 (unused dimensions: box_lo 0, box_n 1); every box keeps at least two
 * parent cells between itself and its parent's edge (HY_EINVAL otherwise).
 * One global step (hy_fmr_step) runs the recursion of the three algorithms:
 * the deepest level steps first, by cfl times its own CFL time step (or by
 * dt_fixed when > 0); every coarser level then steps by the sum of its
 * child's two steps, after a provisional forward-Euler half-step that feeds
 * the child's second step.  Each refined level's exterior (two cells around
 * it) is prolonged from its parent before each step and held through both
 * stages: linear in the primitive variables with minmod-limited parent
 * differences.  After a coarse step the cells just outside the child take the
 * child's fluxes through the shared faces (integrated over its two steps,
 * averaged over the 2^(d-1) fine faces of each coarse face) in place of their
 * own, and the cells under the child become the mean of their children, so
 * mass, momentum and energy summed over the leaf cells change only through
 * the outer boundary.  Device memory: the caller's workspace holds every
 * level (a refined level padded by its exterior) and the flux accumulators. */
#define HY_FMR_MAXLEV 8
typedef struct {
    hy_patch_desc base;
    int nlev;                          /* 1 .. HY_FMR_MAXLEV */
    int64_t box_lo[HY_FMR_MAXLEV][3];  /* entry 0 unused */
    int64_t box_n[HY_FMR_MAXLEV][3];
} hy_fmr_desc;
typedef struct hy_fmr hy_fmr;

hy_status hy_fmr_workspace_bytes(const hy_fmr_desc *d, size_t *bytes);
hy_status hy_fmr_init(const hy_fmr_desc *d, void *dev_workspace, size_t bytes, void *hip_stream, hy_fmr **out);
/* Interior state of one level (nv x that level's cells, FP64 SoA; the
 * exterior of a refined level is filled by prolongation at the next step);
 * synchronising.  HY_EINVAL for a level outside 0 .. nlev - 1; HY_ESTATE as
 * for hy_set_state / hy_get_state. */
hy_status hy_fmr_set_state(hy_fmr *f, int level, int kind, const double *host_soa);
hy_status hy_fmr_get_state(hy_fmr *f, int level, int kind, double *host_soa_out);
/* One global step; *dt_out (may be NULL) receives the coarse step.
 * HY_EINVAL unless solver is HY_HLL or HY_HLLC and cfl > 0 or dt_fixed > 0
 * (finite); HY_ESTATE when a kernel met rho <= 0, p <= 0 or a non-finite
 * value (the levels then hold that step's results).  The
 * levels' times and steps stay in device memory, so the step's launches need
 * no host round trip: they are captured once into a HIP graph per (solver,
 * cfl, dt_fixed) and replayed (hy_fmr_set_graph(f, 0) launches them one by
 * one instead; the results are the same).  Synchronising once, at the end,
 * for the error latches and the coarse step. */
hy_status hy_fmr_step(hy_fmr *f, double cfl, double dt_fixed, int solver, double *dt_out);
hy_status hy_fmr_set_graph(hy_fmr *f, int on);
/* FP64 sums of D, S_x, S_y, S_z, G times the cell volume over the leaf
 * cells of all levels (cells no finer level covers); synchronising. */
hy_status hy_fmr_conserved_totals(hy_fmr *f, double out[5]);
/* hy_autotune on every level (over the cells its stages update: a refined
 * level's interior, in the stage kernel's padded mode; its current state);
 * best, when not NULL, receives nlev shapes.  Results do not change beyond
 * the last-place rounding z chunks can bring.  Drops the captured graph.
 * Synchronising. */
hy_status hy_fmr_autotune(hy_fmr *f, int solver, int reps, hy_launch_cfg *best);
hy_status hy_fmr_destroy(hy_fmr *f);

#ifdef __cplusplus
}
#endif
#endif
