/*
 * FP64 CPU oracle of the single-patch finite-volume hydrodynamics update
 * (Cardall et al., "GenASiS I", Sec. 3).  TEST INFRASTRUCTURE ONLY: it exists
 * to check the GPU library.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the GPU product path never does.
 *
 * Everything is plain double precision, computed in the order the paper
 * states the method: primitive recovery, ghost cells, generalised-minmod
 * slopes (eq. MinMod), face states (eqs. conservedLeft..conservedRight),
 * HLL (eq. FluxHLL) or HLLC (eqs. FluxHLLC, MiddleWaveSpeed, PressureMiddle,
 * EnergyMiddle) fluxes, the cell balance (eq. BalanceEquationAverage) and the
 * two-stage Runge-Kutta step (eqs. RungeKutta1-3) in its literal
 * U^n + (K1 + K2)/2 form.  It shares no source with the GPU library.
 *
 * Arrays are structure-of-arrays, (nv, nz, ny, nx) with x fastest, over
 * interior cells only; nv = ndim + 2.  Conserved order: D, S_1..S_ndim, G.
 * Primitive order: rho, v_1..v_ndim, p.  The baryon mass m is 1, so rho = D.
 */
#ifndef HYDRO_ORACLE_H
#define HYDRO_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ESTATE (-4)   /* rho <= 0, p <= 0 or a non-finite value */

#define ORC_BC_PERIODIC 0
#define ORC_BC_OUTFLOW 1
#define ORC_BC_REFLECT 2

#define ORC_HLL 0
#define ORC_HLLC 1
/* HLLC with HLL at faces transverse to a detected shock (Sec. 3.2 states the
 * switch; the detector is this oracle's reading, see orc_shock_bits) */
#define ORC_HLLC_SWITCH 2
/* shock detector threshold on the relative pressure jump across a cell */
#define ORC_SHOCK_EPS 0.5

#define ORC_LIM_THETA 0
#define ORC_LIM_LEARNED 1

/* learned-limiter network: 4 inputs -> 32 -> 32 -> 1, ReLU */
#define ORC_MLP_IN 4
#define ORC_MLP_H 32
#define ORC_MLP_NPARAM (ORC_MLP_H * ORC_MLP_IN + ORC_MLP_H + ORC_MLP_H * ORC_MLP_H + ORC_MLP_H + ORC_MLP_H + 1)

typedef struct {
    int ndim;          /* 1, 2 or 3 */
    int64_t n[3];      /* interior cells per dimension (unused dims: 1) */
    double lo[3];      /* box corners; cell width (hi - lo) / n */
    double hi[3];
    double gamma;      /* ideal gas p = (gamma - 1) e */
    int bc[3][2];      /* per dimension, low / high face */
    int solver;        /* ORC_HLL, ORC_HLLC or ORC_HLLC_SWITCH */
    int limiter;       /* ORC_LIM_THETA or ORC_LIM_LEARNED */
    double theta;      /* generalised-minmod parameter, 1 <= theta <= 2 */
    double accel[3];   /* uniform acceleration a = -grad(Phi) */
    const double *mlp; /* ORC_MLP_NPARAM parameters when limiter == learned */
    int mlp_bf16;      /* 1: round network operands to bfloat16 first */
    int shock_fp32;    /* 1: the switch's detector compares in FP32 (the
                          precision of an FP32 kernel's decision) */
} orc_desc;

/* Primitive <-> conserved, nv x ncell each.  cons_to_prim returns ORC_ESTATE
 * on a non-physical cell (the output is still written). */
int orc_prim_to_cons(const orc_desc *d, const double *W, double *U);
int orc_cons_to_prim(const orc_desc *d, const double *U, double *W);

/* L(U): the right-hand side of the semi-discrete balance law. */
int orc_rhs(const orc_desc *d, const double *U, double *L);

/* One full two-stage step of size dt, in place. */
int orc_step(const orc_desc *d, double *U, double dt);

/* cfl * min over cells and dimensions of dq / max(|v_q - c|, |v_q + c|). */
int orc_cfl_dt(const orc_desc *d, const double *U, double cfl, double *dt);

/* ---- pointwise pieces, exposed so the tests can pin them ---- */

/* generalised minmod slope from the two one-sided differences */
double orc_limiter_theta(double dm, double dp, double theta);

/* learned slope from a 5-cell stencil w[0..4] centred on w[2] */
double orc_limiter_learned(const double *params, int bf16, const double *w);

/* the network alone on normalised inputs x[4] */
double orc_mlp_forward(const double *params, int bf16, const double *x);

/* Riemann flux at a face normal to dimension q from primitive face states */
void orc_flux(const orc_desc *d, int q, const double *wl, const double *wr, double *f);

/* Physical state of a primitive vector: U, the flux normal to q, and the
 * two outer wave speeds v_q -/+ c. */
void orc_physical(const orc_desc *d, int q, const double *w, double *U, double *F,
                  double *lam_minus, double *lam_plus);

/* Shock flags of every interior cell of U (nz, ny, nx): bit q is set when
 * the pressures of the cell's two neighbours along q (ghost cells by the
 * boundary conditions) differ by more than ORC_SHOCK_EPS times the smaller
 * one and the normal velocity decreases across the cell,
 * v_q(c + e_q) - v_q(c - e_q) < 0 (a compressive jump).  With
 * ORC_HLLC_SWITCH a face normal to r takes the HLL flux when either adjacent
 * cell has a bit q != r set, HLLC otherwise. */
int orc_shock_bits(const orc_desc *d, const double *U, unsigned char *bits);

/* HLLC middle-wave data for the pins: out[0] = alpha_m, out[1] = p*L,
 * out[2] = p*R, then U*L (nv), U*R (nv), F*L (nv), F*R (nv) where the star
 * fluxes come from the jump conditions F* = F_K + s_K (U*_K - U_K). */
void orc_hllc_star(const orc_desc *d, int q, const double *wl, const double *wr, double *out);

/* ---- fixed multilevel refinement (Sec. 2 and Sec. 3.6) ---- */

#define ORC_FMR_MAXLEV 8

/* Level 0 is base (the whole box, its boundary conditions); level l >= 1
 * covers cells box_lo[l] .. box_lo[l] + box_n[l] - 1 of level l - 1, refined
 * by two along every active dimension (unused dimensions: box_lo 0, box_n 1).
 * Each box keeps at least NG = 2 parent cells between itself and the parent
 * level's edge.  HLL or HLLC with the generalised-minmod limiter only. */
typedef struct {
    orc_desc base;
    int nlev;
    int64_t box_lo[ORC_FMR_MAXLEV][3];
    int64_t box_n[ORC_FMR_MAXLEV][3];
    int no_reflux; /* test hook: 1 drops the coarse/fine flux replacement */
} orc_fmr_desc;

/* The descriptor of level l (cells, box corners). */
int orc_fmr_level(const orc_fmr_desc *f, int l, orc_desc *out);

/* Prolongation of the parent level's state into the exterior of level l,
 * linear in the primitive variables with minmod-limited parent differences,
 * stored as conserved variables: Uext has level l's ghosted layout,
 * nv x (n2 + 2NG, n1 + 2NG, n0 + 2NG) over active dimensions; only its ghost
 * cells are written. */
int orc_fmr_prolong(const orc_fmr_desc *f, int l, const double *Uparent, double *Uext);

/* Restriction: every parent cell under level l becomes the mean of its
 * children. */
int orc_fmr_restrict(const orc_fmr_desc *f, int l, const double *Uchild, double *Uparent);

/* One global step (Algs. Evolve / EvolveLevel / StepLevel): U[l] are the
 * levels' interior states, advanced in place to a common time; the deepest
 * level steps by cfl * its CFL time step (or by dt_fixed when > 0), every
 * coarser level by the sum of its child's two steps.  *dt_out receives the
 * coarse step. */
int orc_fmr_step(const orc_fmr_desc *f, double *const *U, double cfl, double dt_fixed, double *dt_out);

/* Host threads for the loops with independent iterations (nthreads <= 0:
 * keep the current count); returns the count in effect (1 without OpenMP).
 * Results do not depend on it. */
int orc_set_threads(int nthreads);

#ifdef __cplusplus
}
#endif
#endif
