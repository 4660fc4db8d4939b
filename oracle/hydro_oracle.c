/*
 * FP64 CPU oracle of the finite-volume hydrodynamics update.  TEST
 * INFRASTRUCTURE ONLY (see hydro_oracle.h).  Plain loops, one step of the
 * method at a time, separate arrays for every intermediate; no blocking,
 * fusion or reordering beyond what the paper's equations state.
 *
 * Loops whose iterations are independent (cells, and lines of cells along a
 * dimension) may run on several host threads (OpenMP); every iteration does
 * the same arithmetic whatever the thread count, so results are bitwise the
 * same on one thread or many.
 */
#include "hydro_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 2 /* ghost layers: the 3-cell generalised-minmod and the 5-cell learned stencil */

static int nvars(const orc_desc *d) { return d->ndim + 2; }

static int64_t ncells(const orc_desc *d) { return d->n[0] * d->n[1] * d->n[2]; }

static double cell_width(const orc_desc *d, int q) { return (d->hi[q] - d->lo[q]) / (double)d->n[q]; }

int orc_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

static int valid_desc(const orc_desc *d)
{
    if (!d || d->ndim < 1 || d->ndim > 3 || !(d->gamma > 1.0)) return 0;
    for (int q = 0; q < 3; ++q) {
        if (d->n[q] < 1) return 0;
        if (q < d->ndim) {
            if (d->n[q] < 2 || !(d->hi[q] > d->lo[q])) return 0;
            for (int s = 0; s < 2; ++s)
                if (d->bc[q][s] < 0 || d->bc[q][s] > 2) return 0;
            if ((d->bc[q][0] == ORC_BC_PERIODIC) != (d->bc[q][1] == ORC_BC_PERIODIC)) return 0;
        } else if (d->n[q] != 1) {
            return 0;
        }
    }
    if (d->limiter == ORC_LIM_LEARNED && !d->mlp) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Fluid variables (Sec. 3.5): D = n, S = m n v, G = e + m n |v|^2 / 2,     */
/* p = (gamma - 1) e from the polytropic closure; m = 1.                    */
/* ------------------------------------------------------------------------ */

static void prim_to_cons_1(int nd, double gamma, const double *w, double *u)
{
    double rho = w[0], p = w[nd + 1], v2 = 0.0;
    for (int r = 0; r < nd; ++r) v2 += w[1 + r] * w[1 + r];
    u[0] = rho;
    for (int r = 0; r < nd; ++r) u[1 + r] = rho * w[1 + r];
    u[nd + 1] = p / (gamma - 1.0) + 0.5 * rho * v2;
}

static int cons_to_prim_1(int nd, double gamma, const double *u, double *w)
{
    double D = u[0], s2 = 0.0;
    w[0] = D;
    for (int r = 0; r < nd; ++r) {
        w[1 + r] = u[1 + r] / D;
        s2 += u[1 + r] * u[1 + r];
    }
    double e = u[nd + 1] - 0.5 * s2 / D;
    w[nd + 1] = (gamma - 1.0) * e;
    int ok = (w[0] > 0.0) && (w[nd + 1] > 0.0) && isfinite(w[0]) && isfinite(w[nd + 1]);
    for (int r = 0; r < nd; ++r) ok = ok && isfinite(w[1 + r]);
    return ok;
}

int orc_prim_to_cons(const orc_desc *d, const double *W, double *U)
{
    if (!valid_desc(d)) return ORC_EINVAL;
    int nv = nvars(d);
    int64_t N = ncells(d);
    double w[5], u[5];
    for (int64_t c = 0; c < N; ++c) {
        for (int v = 0; v < nv; ++v) w[v] = W[v * N + c];
        prim_to_cons_1(d->ndim, d->gamma, w, u);
        for (int v = 0; v < nv; ++v) U[v * N + c] = u[v];
    }
    return ORC_OK;
}

int orc_cons_to_prim(const orc_desc *d, const double *U, double *W)
{
    if (!valid_desc(d)) return ORC_EINVAL;
    int nv = nvars(d);
    int64_t N = ncells(d);
    int status = ORC_OK;
    double w[5], u[5];
    for (int64_t c = 0; c < N; ++c) {
        for (int v = 0; v < nv; ++v) u[v] = U[v * N + c];
        if (!cons_to_prim_1(d->ndim, d->gamma, u, w)) status = ORC_ESTATE;
        for (int v = 0; v < nv; ++v) W[v * N + c] = w[v];
    }
    return status;
}

/* Physical flux normal to q (eqs. FluxBaryon, FluxMomentumFluid and the
 * energy flux) and the outer wave speeds v_q -/+ c_s, c_s = sqrt(gamma p / rho). */
void orc_physical(const orc_desc *d, int q, const double *w, double *U, double *F,
                  double *lam_minus, double *lam_plus)
{
    int nd = d->ndim;
    prim_to_cons_1(nd, d->gamma, w, U);
    double rho = w[0], p = w[nd + 1], vq = w[1 + q];
    F[0] = rho * vq;
    for (int r = 0; r < nd; ++r) F[1 + r] = rho * w[1 + r] * vq + (r == q ? p : 0.0);
    F[nd + 1] = (U[nd + 1] + p) * vq; /* (e + p + rho |v|^2 / 2) v_q */
    double cs = sqrt(d->gamma * p / rho);
    *lam_minus = vq - cs;
    *lam_plus = vq + cs;
}

/* ------------------------------------------------------------------------ */
/* Riemann solvers (Sec. 3.2 and 3.5)                                       */
/* ------------------------------------------------------------------------ */

static double max3(double a, double b, double c) { return fmax(a, fmax(b, c)); }

/* Davis-type outer speeds: alpha_+/- = max(0, +/-lambda_+/-(U_L), +/-lambda_+/-(U_R)). */
static void outer_speeds(double lmL, double lpL, double lmR, double lpR, double *ap, double *am)
{
    *ap = max3(0.0, lpL, lpR);
    *am = max3(0.0, -lmL, -lmR);
}

/* HLLC middle states for side K (0 = left, 1 = right) from the jump
 * conditions across the outer wave s_K (s_L = -alpha_-, s_R = +alpha_+):
 *   rho*_K = rho_K (s_K - v_K) / (s_K - alpha_m)
 *   p*_K   = p_K + rho_K (s_K - v_K)(alpha_m - v_K)
 *   G*_K   = [(s_K - v_K) G_K - p_K v_K + p*_K alpha_m] / (s_K - alpha_m)
 * with the normal velocity alpha_m and unchanged transverse velocities.  The
 * printed pressure and energy relations carry a sign slip and a starred G on
 * the right-hand side; these are the forms the jump conditions give. */
static void hllc_side(const orc_desc *d, int q, const double *w, const double *U, double sK,
                      double am_, double *Ustar, double *pstar)
{
    int nd = d->ndim;
    double rho = w[0], vK = w[1 + q], pK = w[nd + 1], GK = U[nd + 1];
    double rs = rho * (sK - vK) / (sK - am_);
    double ps = pK + rho * (sK - vK) * (am_ - vK);
    double Gs = ((sK - vK) * GK - pK * vK + ps * am_) / (sK - am_);
    Ustar[0] = rs;
    for (int r = 0; r < nd; ++r) Ustar[1 + r] = (r == q) ? rs * am_ : rs * w[1 + r];
    Ustar[nd + 1] = Gs;
    *pstar = ps;
}

/* Batten's middle-wave speed, eq. MiddleWaveSpeed: S_HLL / (m D_HLL). */
static double middle_speed(int nd, int q, const double *wl, const double *wr, double ap, double am)
{
    double rl = wl[0], vl = wl[1 + q], pl = wl[nd + 1];
    double rr = wr[0], vr = wr[1 + q], pr = wr[nd + 1];
    double num = rr * vr * (ap - vr) + rl * vl * (am + vl) - (pr - pl);
    double den = rr * (ap - vr) + rl * (am + vl);
    return num / den;
}

void orc_flux(const orc_desc *d, int q, const double *wl, const double *wr, double *f)
{
    int nv = nvars(d);
    double UL[5], FL[5], UR[5], FR[5], lmL, lpL, lmR, lpR, ap, am;
    orc_physical(d, q, wl, UL, FL, &lmL, &lpL);
    orc_physical(d, q, wr, UR, FR, &lmR, &lpR);
    outer_speeds(lmL, lpL, lmR, lpR, &ap, &am);
    if (d->solver == ORC_HLL) {
        /* eq. FluxHLL; both speeds vanish only for c = 0 on both sides */
        if (ap + am > 0.0) {
            for (int v = 0; v < nv; ++v)
                f[v] = (ap * FL[v] + am * FR[v] - ap * am * (UR[v] - UL[v])) / (ap + am);
        } else {
            for (int v = 0; v < nv; ++v) f[v] = 0.5 * (FL[v] + FR[v]);
        }
        return;
    }
    /* eq. FluxHLLC, cases tested in the printed order */
    if (am == 0.0) {
        for (int v = 0; v < nv; ++v) f[v] = FL[v];
        return;
    }
    if (ap == 0.0) {
        for (int v = 0; v < nv; ++v) f[v] = FR[v];
        return;
    }
    double a_m = middle_speed(d->ndim, q, wl, wr, ap, am);
    double Us[5], ps;
    if (a_m >= 0.0) {
        double sL = -am;
        hllc_side(d, q, wl, UL, sL, a_m, Us, &ps);
        for (int v = 0; v < nv; ++v) f[v] = FL[v] + sL * (Us[v] - UL[v]);
    } else {
        double sR = ap;
        hllc_side(d, q, wr, UR, sR, a_m, Us, &ps);
        for (int v = 0; v < nv; ++v) f[v] = FR[v] + sR * (Us[v] - UR[v]);
    }
}

void orc_hllc_star(const orc_desc *d, int q, const double *wl, const double *wr, double *out)
{
    int nv = nvars(d);
    double UL[5], FL[5], UR[5], FR[5], lmL, lpL, lmR, lpR, ap, am;
    orc_physical(d, q, wl, UL, FL, &lmL, &lpL);
    orc_physical(d, q, wr, UR, FR, &lmR, &lpR);
    outer_speeds(lmL, lpL, lmR, lpR, &ap, &am);
    double a_m = middle_speed(d->ndim, q, wl, wr, ap, am);
    double UsL[5], UsR[5], psL, psR;
    hllc_side(d, q, wl, UL, -am, a_m, UsL, &psL);
    hllc_side(d, q, wr, UR, ap, a_m, UsR, &psR);
    out[0] = a_m;
    out[1] = psL;
    out[2] = psR;
    for (int v = 0; v < nv; ++v) {
        out[3 + v] = UsL[v];
        out[3 + nv + v] = UsR[v];
        out[3 + 2 * nv + v] = FL[v] - am * (UsL[v] - UL[v]);
        out[3 + 3 * nv + v] = FR[v] + ap * (UsR[v] - UR[v]);
    }
}

/* ------------------------------------------------------------------------ */
/* Slope limiters                                                           */
/* ------------------------------------------------------------------------ */

/* MM: the argument of smallest magnitude if all three share a sign, else 0. */
static double minmod3(double a, double b, double c)
{
    if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
    if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
    return 0.0;
}

/* eq. MinMod on a uniform grid, as a per-cell difference:
 * sigma = MM(theta dm, (dm + dp) / 2, theta dp). */
double orc_limiter_theta(double dm, double dp, double theta)
{
    return minmod3(theta * dm, 0.5 * (dm + dp), theta * dp);
}

/* round to the nearest bfloat16 (ties to even) through binary32 */
static double to_bf16(double x)
{
    float f = (float)x;
    uint32_t b;
    memcpy(&b, &f, 4);
    if ((b & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan unchanged */
    b += 0x7fffu + ((b >> 16) & 1u);
    b &= 0xffff0000u;
    memcpy(&f, &b, 4);
    return (double)f;
}

/* Parameters: W1[32][4], b1[32], W2[32][32], b2[32], w3[32], b3.
 * h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3.
 * With bf16 set, the operands of all three layers are rounded to bfloat16
 * (x, W1, h1, W2, h2, w3); biases, b3 and all arithmetic stay double. */
double orc_mlp_forward(const double *P, int bf16, const double *x)
{
    const double *W1 = P, *b1 = W1 + ORC_MLP_H * ORC_MLP_IN, *W2 = b1 + ORC_MLP_H;
    const double *b2 = W2 + ORC_MLP_H * ORC_MLP_H, *w3 = b2 + ORC_MLP_H, *b3 = w3 + ORC_MLP_H;
    double xi[ORC_MLP_IN], h1[ORC_MLP_H], h2[ORC_MLP_H];
    for (int k = 0; k < ORC_MLP_IN; ++k) xi[k] = bf16 ? to_bf16(x[k]) : x[k];
    for (int j = 0; j < ORC_MLP_H; ++j) {
        double s = 0.0;
        for (int k = 0; k < ORC_MLP_IN; ++k) {
            double wjk = W1[j * ORC_MLP_IN + k];
            s += (bf16 ? to_bf16(wjk) : wjk) * xi[k];
        }
        s += b1[j];
        h1[j] = s > 0.0 ? s : 0.0;
        if (bf16) h1[j] = to_bf16(h1[j]);
    }
    for (int j = 0; j < ORC_MLP_H; ++j) {
        double s = 0.0;
        for (int k = 0; k < ORC_MLP_H; ++k) {
            double wjk = W2[j * ORC_MLP_H + k];
            s += (bf16 ? to_bf16(wjk) : wjk) * h1[k];
        }
        s += b2[j];
        h2[j] = s > 0.0 ? s : 0.0;
        if (bf16) h2[j] = to_bf16(h2[j]);
    }
    double y = b3[0];
    for (int k = 0; k < ORC_MLP_H; ++k) y += (bf16 ? to_bf16(w3[k]) : w3[k]) * h2[k];
    return y;
}

/* Learned slope from w[0..4]: inputs are the four one-sided differences over
 * s = max|d| + 1e-12 (|w_2| + 1e-30); the network output times s is clamped
 * to the TVD region 0 <= sign(D) sigma <= 2 min(|D-|, |D+|), and to 0 where
 * the two central differences D- = d2, D+ = d3 disagree in sign. */
double orc_limiter_learned(const double *params, int bf16, const double *w)
{
    double dlt[4];
    for (int k = 0; k < 4; ++k) dlt[k] = w[k + 1] - w[k];
    double s = 0.0;
    for (int k = 0; k < 4; ++k) s = fmax(s, fabs(dlt[k]));
    s += 1e-12 * (fabs(w[2]) + 1e-30);
    double x[4];
    for (int k = 0; k < 4; ++k) x[k] = dlt[k] / s;
    double sigma = s * orc_mlp_forward(params, bf16, x);
    double dm = dlt[1], dp = dlt[2];
    if (dm * dp <= 0.0) return 0.0;
    double lim = 2.0 * fmin(fabs(dm), fabs(dp));
    double sg = dp > 0.0 ? 1.0 : -1.0;
    return sg * fmin(fmax(sg * sigma, 0.0), lim);
}

/* ------------------------------------------------------------------------ */
/* Ghost cells (reading of Alg. 1 line 7): ng layers filled from cell-centre */
/* primitives; periodic wraps, outflow copies the nearest interior cell,    */
/* reflecting mirrors and negates the normal velocity.                      */
/* ------------------------------------------------------------------------ */

static int64_t map_coord(int64_t i, int64_t n, const int *bc, int *flip)
{
    if (i < 0) {
        if (bc[0] == ORC_BC_PERIODIC) return ((i % n) + n) % n;
        if (bc[0] == ORC_BC_OUTFLOW) return 0;
        *flip = 1;
        int64_t m = -1 - i;
        return m < n ? m : n - 1;
    }
    if (i >= n) {
        if (bc[1] == ORC_BC_PERIODIC) return i % n;
        if (bc[1] == ORC_BC_OUTFLOW) return n - 1;
        *flip = 1;
        int64_t m = 2 * n - 1 - i;
        return m >= 0 ? m : 0;
    }
    return i;
}

typedef struct {
    int64_t m[3]; /* ghosted extents */
    int64_t g[3]; /* ghost layers per dim (NG on active dims, 0 otherwise) */
} ghost_geom;

static ghost_geom make_geom(const orc_desc *d)
{
    ghost_geom G;
    for (int q = 0; q < 3; ++q) {
        G.g[q] = q < d->ndim ? NG : 0;
        G.m[q] = d->n[q] + 2 * G.g[q];
    }
    return G;
}

static int64_t gidx(const ghost_geom *G, int64_t i, int64_t j, int64_t k)
{
    return ((k + G->g[2]) * G->m[1] + (j + G->g[1])) * G->m[0] + (i + G->g[0]);
}

/* Interior primitives into the ghosted array, then every ghost cell from its
 * mapped interior source, or, when Uext is given (a refined level, whose
 * exterior comes from the next coarser level), from the conserved values Uext
 * holds at that ghost cell (ghosted layout). */
static int fill_primitives(const orc_desc *d, const double *U, const double *Uext, const ghost_geom *G, double *Wg)
{
    int nd = d->ndim, nv = nvars(d);
    int64_t N = ncells(d), M = G->m[0] * G->m[1] * G->m[2];
    int status = ORC_OK;
#pragma omp parallel for schedule(static) reduction(min : status)
    for (int64_t k = 0; k < d->n[2]; ++k)
        for (int64_t j = 0; j < d->n[1]; ++j)
            for (int64_t i = 0; i < d->n[0]; ++i) {
                double u[5], w[5];
                int64_t c = (k * d->n[1] + j) * d->n[0] + i;
                for (int v = 0; v < nv; ++v) u[v] = U[v * N + c];
                if (!cons_to_prim_1(nd, d->gamma, u, w)) status = ORC_ESTATE;
                int64_t g = gidx(G, i, j, k);
                for (int v = 0; v < nv; ++v) Wg[v * M + g] = w[v];
            }
    /* ghosts read interior cells only, so the planes are independent */
#pragma omp parallel for schedule(static) reduction(min : status)
    for (int64_t k = -G->g[2]; k < d->n[2] + G->g[2]; ++k)
        for (int64_t j = -G->g[1]; j < d->n[1] + G->g[1]; ++j)
            for (int64_t i = -G->g[0]; i < d->n[0] + G->g[0]; ++i) {
                double u[5], w[5];
                int inside = i >= 0 && i < d->n[0] && j >= 0 && j < d->n[1] && k >= 0 && k < d->n[2];
                if (inside) continue;
                if (Uext) {
                    int64_t g = gidx(G, i, j, k);
                    for (int v = 0; v < nv; ++v) u[v] = Uext[v * M + g];
                    if (!cons_to_prim_1(nd, d->gamma, u, w)) status = ORC_ESTATE;
                    for (int v = 0; v < nv; ++v) Wg[v * M + g] = w[v];
                    continue;
                }
                int flip[3] = {0, 0, 0};
                int64_t si = map_coord(i, d->n[0], d->bc[0], &flip[0]);
                int64_t sj = nd > 1 ? map_coord(j, d->n[1], d->bc[1], &flip[1]) : 0;
                int64_t sk = nd > 2 ? map_coord(k, d->n[2], d->bc[2], &flip[2]) : 0;
                int64_t src = gidx(G, si, sj, sk), dst = gidx(G, i, j, k);
                for (int v = 0; v < nv; ++v) Wg[v * M + dst] = Wg[v * M + src];
                for (int q = 0; q < nd; ++q)
                    if (flip[q]) Wg[(1 + q) * M + dst] = -Wg[(1 + q) * M + dst];
            }
    return status;
}

/* ------------------------------------------------------------------------ */
/* Shock detector for the HLLC -> HLL switch.  Sec. 3.2 says HLL replaces    */
/* HLLC in the immediate vicinity of a shock, in the directions transverse  */
/* to its propagation, against odd-even decoupling, without giving the      */
/* detector.  Reading: a cell is in a shock moving along q when the         */
/* pressures on its two sides along q differ by more than ORC_SHOCK_EPS of  */
/* the smaller one and the flow converges there; a face normal to r is in   */
/* the vicinity of a shock transverse to it when one of its two cells is    */
/* flagged along a direction q != r.                                        */
/* ------------------------------------------------------------------------ */

/* flag bits of the cell at ghosted coordinates (i, j, k); every neighbour
 * along an active dimension must lie inside the ghosted array */
static unsigned cell_shock_bits(const orc_desc *d, const ghost_geom *G, const double *Wg, int64_t i, int64_t j,
                                int64_t k)
{
    int nd = d->ndim;
    int64_t M = G->m[0] * G->m[1] * G->m[2];
    unsigned bits = 0;
    for (int q = 0; q < nd; ++q) {
        int64_t lo3[3] = {i, j, k}, hi3[3] = {i, j, k};
        lo3[q] -= 1;
        hi3[q] += 1;
        int64_t a = gidx(G, lo3[0], lo3[1], lo3[2]), b = gidx(G, hi3[0], hi3[1], hi3[2]);
        double pa = Wg[(nd + 1) * M + a], pb = Wg[(nd + 1) * M + b];
        double va = Wg[(1 + q) * M + a], vb = Wg[(1 + q) * M + b];
        if (d->shock_fp32) {
            /* the decision in the precision an FP32 kernel takes it */
            float fpa = (float)pa, fpb = (float)pb, fva = (float)va, fvb = (float)vb;
            if (fabsf(fpb - fpa) > (float)ORC_SHOCK_EPS * fminf(fpa, fpb) && fvb - fva < 0.0f) bits |= 1u << q;
        } else if (fabs(pb - pa) > ORC_SHOCK_EPS * fmin(pa, pb) && vb - va < 0.0) {
            bits |= 1u << q;
        }
    }
    return bits;
}

int orc_shock_bits(const orc_desc *d, const double *U, unsigned char *bits)
{
    if (!valid_desc(d) || !bits) return ORC_EINVAL;
    ghost_geom G = make_geom(d);
    int64_t M = G.m[0] * G.m[1] * G.m[2];
    double *Wg = (double *)malloc(sizeof(double) * nvars(d) * M);
    if (!Wg) return ORC_EINVAL;
    int status = fill_primitives(d, U, NULL, &G, Wg);
    for (int64_t k = 0; k < d->n[2]; ++k)
        for (int64_t j = 0; j < d->n[1]; ++j)
            for (int64_t i = 0; i < d->n[0]; ++i)
                bits[(k * d->n[1] + j) * d->n[0] + i] = (unsigned char)cell_shock_bits(d, &G, Wg, i, j, k);
    free(Wg);
    return status;
}

/* ------------------------------------------------------------------------ */
/* The semi-discrete right-hand side, eq. BalanceEquationAverage on a        */
/* Cartesian grid: L = -sum_q (F_{i+1/2} - F_{i-1/2}) / dq + S.              */
/* ------------------------------------------------------------------------ */

/* Face fluxes a multilevel step needs (Alg. StepLevel): own[q][s] receives
 * the fluxes through the level's own low (s = 0) and high (s = 1) boundary
 * faces normal to q, child[q][s] those through the faces of the box of cells
 * the next finer level covers.  Layout nv x (t2, t1), t1 the index along
 * dimension (q + 1) % 3 and t2 along (q + 2) % 3, over the level's cells
 * (own) or the box's cells (child).  NULL pointers are skipped. */
typedef struct {
    double *own[3][2];
    double *child[3][2];
    int64_t clo[3], cn[3]; /* the child box, in this level's cells */
} face_rec;

static int rhs_core(const orc_desc *d, const double *U, const double *Uext, double *L, face_rec *rec)
{
    if (!valid_desc(d)) return ORC_EINVAL;
    int nd = d->ndim, nv = nvars(d);
    int64_t N = ncells(d);
    ghost_geom G = make_geom(d);
    int64_t M = G.m[0] * G.m[1] * G.m[2];
    double *Wg = (double *)malloc(sizeof(double) * nv * M);
    if (!Wg) return ORC_EINVAL;
    int status = fill_primitives(d, U, Uext, &G, Wg);

    /* sources: S = (0, rho a, rho v . a) for a uniform acceleration a */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        L[c] = 0.0;
        double power = 0.0;
        for (int r = 0; r < nd; ++r) {
            L[(1 + r) * N + c] = U[c] * d->accel[r];
            power += U[(1 + r) * N + c] * d->accel[r];
        }
        L[(nd + 1) * N + c] = power;
    }

    for (int q = 0; q < nd; ++q) {
        int64_t nq = d->n[q];
        double dq = cell_width(d, q);
        /* one line along q at a time; the line holds cells -NG .. nq+NG-1.
         * Lines are independent (each writes L only at its own cells). */
        int64_t len = nq + 2 * NG;
        int64_t t1n = d->n[(q + 1) % 3], t2n = d->n[(q + 2) % 3];
#pragma omp parallel
        {
        double *wl = (double *)malloc(sizeof(double) * nv * len);
        double *sig = (double *)malloc(sizeof(double) * nv * (nq + 2)); /* cells -1 .. nq */
        double *F = (double *)malloc(sizeof(double) * nv * (nq + 1));   /* faces -1/2 .. nq-1/2 */
#pragma omp for collapse(2) schedule(static)
        for (int64_t b = 0; b < t2n; ++b)
            for (int64_t a = 0; a < t1n; ++a) {
                int64_t idx3[3];
                for (int64_t s = -NG; s < nq + NG; ++s) {
                    idx3[q] = s;
                    idx3[(q + 1) % 3] = a;
                    idx3[(q + 2) % 3] = b;
                    int64_t g = gidx(&G, idx3[0], idx3[1], idx3[2]);
                    for (int v = 0; v < nv; ++v) wl[v * len + (s + NG)] = Wg[v * M + g];
                }
                /* slopes (per cell differences) for cells -1 .. nq */
                for (int v = 0; v < nv; ++v) {
                    const double *line = wl + v * len + NG; /* line[s] = cell s */
                    if (d->limiter == ORC_LIM_THETA) {
                        for (int64_t s = -1; s <= nq; ++s)
                            sig[v * (nq + 2) + (s + 1)] =
                                orc_limiter_theta(line[s] - line[s - 1], line[s + 1] - line[s], d->theta);
                    } else {
                        for (int64_t s = 0; s < nq; ++s)
                            sig[v * (nq + 2) + (s + 1)] = orc_limiter_learned(d->mlp, d->mlp_bf16, line + s - 2);
                        /* boundary conditions applied to reconstructed values:
                         * the ghost slope comes from the mapped interior cell */
                        double lo_s, hi_s;
                        if (d->bc[q][0] == ORC_BC_PERIODIC) {
                            lo_s = sig[v * (nq + 2) + nq];
                            hi_s = sig[v * (nq + 2) + 1];
                        } else {
                            double par = (v == 1 + q) ? 1.0 : -1.0;
                            lo_s = d->bc[q][0] == ORC_BC_REFLECT ? par * sig[v * (nq + 2) + 1] : 0.0;
                            hi_s = d->bc[q][1] == ORC_BC_REFLECT ? par * sig[v * (nq + 2) + nq] : 0.0;
                        }
                        sig[v * (nq + 2) + 0] = lo_s;
                        sig[v * (nq + 2) + nq + 1] = hi_s;
                    }
                }
                /* face f sits between cells f-1 and f: left state is the
                 * outer face value of cell f-1, right state the inner face
                 * value of cell f */
                for (int64_t f = 0; f <= nq; ++f) {
                    double wlft[5], wrgt[5], flx[5];
                    for (int v = 0; v < nv; ++v) {
                        const double *line = wl + v * len + NG;
                        wlft[v] = line[f - 1] + 0.5 * sig[v * (nq + 2) + f];
                        wrgt[v] = line[f] - 0.5 * sig[v * (nq + 2) + f + 1];
                    }
                    if (d->solver == ORC_HLLC_SWITCH) {
                        /* cells f-1 and f along q, at the line's transverse position */
                        int64_t cl[3], cr[3];
                        cl[q] = f - 1;
                        cr[q] = f;
                        cl[(q + 1) % 3] = cr[(q + 1) % 3] = a;
                        cl[(q + 2) % 3] = cr[(q + 2) % 3] = b;
                        unsigned fl_bits = cell_shock_bits(d, &G, Wg, cl[0], cl[1], cl[2]);
                        unsigned fr_bits = cell_shock_bits(d, &G, Wg, cr[0], cr[1], cr[2]);
                        orc_desc dd = *d;
                        dd.solver = ((fl_bits | fr_bits) & ~(1u << q)) ? ORC_HLL : ORC_HLLC;
                        orc_flux(&dd, q, wlft, wrgt, flx);
                    } else {
                        orc_flux(d, q, wlft, wrgt, flx);
                    }
                    for (int v = 0; v < nv; ++v) F[v * (nq + 1) + f] = flx[v];
                }
                if (rec) {
                    int64_t t = b * t1n + a;
                    for (int v = 0; v < nv; ++v) {
                        if (rec->own[q][0]) rec->own[q][0][v * t1n * t2n + t] = F[v * (nq + 1) + 0];
                        if (rec->own[q][1]) rec->own[q][1][v * t1n * t2n + t] = F[v * (nq + 1) + nq];
                    }
                    int r1 = (q + 1) % 3, r2 = (q + 2) % 3;
                    int64_t ca = a - rec->clo[r1], cb = b - rec->clo[r2];
                    if (rec->child[q][0] && ca >= 0 && ca < rec->cn[r1] && cb >= 0 && cb < rec->cn[r2]) {
                        int64_t ct = cb * rec->cn[r1] + ca, cnt = rec->cn[r1] * rec->cn[r2];
                        for (int v = 0; v < nv; ++v) {
                            rec->child[q][0][v * cnt + ct] = F[v * (nq + 1) + rec->clo[q]];
                            rec->child[q][1][v * cnt + ct] = F[v * (nq + 1) + rec->clo[q] + rec->cn[q]];
                        }
                    }
                }
                for (int64_t s = 0; s < nq; ++s) {
                    idx3[q] = s;
                    idx3[(q + 1) % 3] = a;
                    idx3[(q + 2) % 3] = b;
                    int64_t c = (idx3[2] * d->n[1] + idx3[1]) * d->n[0] + idx3[0];
                    for (int v = 0; v < nv; ++v)
                        L[v * N + c] -= (F[v * (nq + 1) + s + 1] - F[v * (nq + 1) + s]) / dq;
                }
            }
        free(wl);
        free(sig);
        free(F);
        }
    }
    free(Wg);
    return status;
}

int orc_rhs(const orc_desc *d, const double *U, double *L) { return rhs_core(d, U, NULL, L, NULL); }

/* eqs. Update and RungeKutta1-3: K1 = dt L(U^n), U1 = U^n + K1,
 * K2 = dt L(U1), U^{n+1} = U^n + (K1 + K2) / 2. */
int orc_step(const orc_desc *d, double *U, double dt)
{
    if (!valid_desc(d) || !(dt > 0.0) || !isfinite(dt)) return ORC_EINVAL;
    int nv = nvars(d);
    int64_t T = nv * ncells(d);
    double *L = (double *)malloc(sizeof(double) * T);
    double *K1 = (double *)malloc(sizeof(double) * T);
    double *U1 = (double *)malloc(sizeof(double) * T);
    int s1 = orc_rhs(d, U, L);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < T; ++i) {
        K1[i] = dt * L[i];
        U1[i] = U[i] + K1[i];
    }
    int s2 = orc_rhs(d, U1, L);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < T; ++i) {
        double K2 = dt * L[i];
        U[i] = U[i] + 0.5 * (K1[i] + K2);
    }
    free(L);
    free(K1);
    free(U1);
    if (s1 != ORC_OK) return s1;
    return s2;
}

/* eq. courantTimeStep times the Courant factor. */
int orc_cfl_dt(const orc_desc *d, const double *U, double cfl, double *dt)
{
    if (!valid_desc(d)) return ORC_EINVAL;
    int nd = d->ndim, nv = nvars(d);
    int64_t N = ncells(d);
    int status = ORC_OK;
    double m = INFINITY, u[5], w[5];
    for (int64_t c = 0; c < N; ++c) {
        for (int v = 0; v < nv; ++v) u[v] = U[v * N + c];
        if (!cons_to_prim_1(nd, d->gamma, u, w)) status = ORC_ESTATE;
        double cs = sqrt(d->gamma * w[nd + 1] / w[0]);
        for (int q = 0; q < nd; ++q) {
            double lm = w[1 + q] - cs, lp = w[1 + q] + cs;
            double t = cell_width(d, q) / fmax(fabs(lm), fabs(lp));
            if (t < m) m = t;
        }
    }
    *dt = cfl * m;
    return status;
}

/* ------------------------------------------------------------------------ */
/* Fixed multilevel refinement: nested levels, each a box of cells of the   */
/* next coarser level refined by two in every active dimension (Sec. 2, the */
/* refinable mesh), stepped with subcycling and conservative coarse/fine    */
/* flux replacement (Sec. 3.6, Algs. Evolve, EvolveLevel and StepLevel).   */
/* Readings where the paper leaves the detail open:                         */
/*  - prolongation only ever fills a level's exterior, so it need not      */
/*    conserve: it is linear in the primitive variables with minmod-limited */
/*    per-dimension differences of the parent (the limited option of the    */
/*    paper's footnote), which keeps density and pressure positive next to  */
/*    strong shocks; a child at offset +-1/4 of the parent width along q    */
/*    takes W_p +- sigma_q / 4.  Restriction is the mean of the children's  */
/*    conserved variables.                                                  */
/*  - a refined level's exterior (ng cells around it) is prolonged once per */
/*    step and held fixed through both Runge-Kutta stages;                  */
/*  - before the provisional step of a refined coarse level its exterior is */
/*    prolonged from its own parent as it stands (the same data the full   */
/*    step then uses);                                                      */
/*  - the coarse/fine replacement acts on the step's net update: the coarse */
/*    cell outside the child box gets the difference between the fine       */
/*    fluxes, integrated over both fine steps and averaged over the fine    */
/*    faces of the coarse face, and its own flux integrated over the step.  */
/* ------------------------------------------------------------------------ */

static int fmr_valid(const orc_fmr_desc *f)
{
    if (!f || f->nlev < 1 || f->nlev > ORC_FMR_MAXLEV || !valid_desc(&f->base)) return 0;
    if (f->base.solver != ORC_HLL && f->base.solver != ORC_HLLC) return 0;
    if (f->base.limiter != ORC_LIM_THETA) return 0;
    int64_t n[3] = {f->base.n[0], f->base.n[1], f->base.n[2]};
    for (int l = 1; l < f->nlev; ++l)
        for (int q = 0; q < 3; ++q) {
            if (q < f->base.ndim) {
                if (f->box_n[l][q] < 1 || f->box_lo[l][q] < NG || f->box_lo[l][q] + f->box_n[l][q] > n[q] - NG)
                    return 0;
                n[q] = 2 * f->box_n[l][q];
            } else if (f->box_lo[l][q] != 0 || f->box_n[l][q] != 1) {
                return 0;
            }
        }
    return 1;
}

int orc_fmr_level(const orc_fmr_desc *f, int l, orc_desc *out)
{
    if (!fmr_valid(f) || l < 0 || l >= f->nlev || !out) return ORC_EINVAL;
    orc_desc d = f->base;
    for (int k = 1; k <= l; ++k)
        for (int q = 0; q < d.ndim; ++q) {
            double dq = cell_width(&d, q);
            d.lo[q] = d.lo[q] + (double)f->box_lo[k][q] * dq;
            d.hi[q] = d.lo[q] + (double)f->box_n[k][q] * dq;
            d.n[q] = 2 * f->box_n[k][q];
            /* the exterior is supplied by prolongation; the kinds are unused */
            d.bc[q][0] = d.bc[q][1] = ORC_BC_OUTFLOW;
        }
    *out = d;
    return ORC_OK;
}

static int64_t floor_half(int64_t i) { return i >= 0 ? i / 2 : -((-i + 1) / 2); }

int orc_fmr_prolong(const orc_fmr_desc *f, int l, const double *Uparent, double *Uext)
{
    if (!fmr_valid(f) || l < 1 || l >= f->nlev || !Uparent || !Uext) return ORC_EINVAL;
    orc_desc pd, cd;
    orc_fmr_level(f, l - 1, &pd);
    orc_fmr_level(f, l, &cd);
    int nd = cd.ndim, nv = nvars(&cd);
    int64_t NP = ncells(&pd);
    ghost_geom G = make_geom(&cd);
    int64_t M = G.m[0] * G.m[1] * G.m[2];
    int status = ORC_OK;
    for (int64_t k = -G.g[2]; k < cd.n[2] + G.g[2]; ++k)
        for (int64_t j = -G.g[1]; j < cd.n[1] + G.g[1]; ++j)
            for (int64_t i = -G.g[0]; i < cd.n[0] + G.g[0]; ++i) {
                int inside = i >= 0 && i < cd.n[0] && j >= 0 && j < cd.n[1] && k >= 0 && k < cd.n[2];
                if (inside) continue;
                int64_t c3[3] = {i, j, k}, p3[3], s3[3];
                for (int q = 0; q < 3; ++q) {
                    if (q < nd) {
                        p3[q] = f->box_lo[l][q] + floor_half(c3[q]);
                        s3[q] = c3[q] - 2 * floor_half(c3[q]);
                    } else {
                        p3[q] = 0;
                        s3[q] = 0;
                    }
                }
                /* the parent and its two neighbours along each active q, in
                 * primitive variables */
                double w0[5], wm[3][5], wp[3][5], u[5], wc[5];
                int64_t pc = (p3[2] * pd.n[1] + p3[1]) * pd.n[0] + p3[0];
                for (int v = 0; v < nv; ++v) u[v] = Uparent[v * NP + pc];
                if (!cons_to_prim_1(nd, cd.gamma, u, w0)) status = ORC_ESTATE;
                for (int q = 0; q < nd; ++q) {
                    int64_t lo3[3] = {p3[0], p3[1], p3[2]}, hi3[3] = {p3[0], p3[1], p3[2]};
                    lo3[q] -= 1;
                    hi3[q] += 1;
                    int64_t cm = (lo3[2] * pd.n[1] + lo3[1]) * pd.n[0] + lo3[0];
                    int64_t cp = (hi3[2] * pd.n[1] + hi3[1]) * pd.n[0] + hi3[0];
                    for (int v = 0; v < nv; ++v) u[v] = Uparent[v * NP + cm];
                    if (!cons_to_prim_1(nd, cd.gamma, u, wm[q])) status = ORC_ESTATE;
                    for (int v = 0; v < nv; ++v) u[v] = Uparent[v * NP + cp];
                    if (!cons_to_prim_1(nd, cd.gamma, u, wp[q])) status = ORC_ESTATE;
                }
                for (int v = 0; v < nv; ++v) {
                    double val = w0[v];
                    for (int q = 0; q < nd; ++q) {
                        double sigma = orc_limiter_theta(w0[v] - wm[q][v], wp[q][v] - w0[v], 1.0);
                        val += (s3[q] ? 0.25 : -0.25) * sigma;
                    }
                    wc[v] = val;
                }
                prim_to_cons_1(nd, cd.gamma, wc, u);
                int64_t g = gidx(&G, i, j, k);
                for (int v = 0; v < nv; ++v) Uext[v * M + g] = u[v];
            }
    return status;
}

int orc_fmr_restrict(const orc_fmr_desc *f, int l, const double *Uchild, double *Uparent)
{
    if (!fmr_valid(f) || l < 1 || l >= f->nlev || !Uparent || !Uchild) return ORC_EINVAL;
    orc_desc pd, cd;
    orc_fmr_level(f, l - 1, &pd);
    orc_fmr_level(f, l, &cd);
    int nd = cd.ndim, nv = nvars(&cd);
    int64_t NP = ncells(&pd), NC = ncells(&cd);
    int nchild = 1 << nd;
    for (int64_t k = 0; k < f->box_n[l][2]; ++k)
        for (int64_t j = 0; j < f->box_n[l][1]; ++j)
            for (int64_t i = 0; i < f->box_n[l][0]; ++i) {
                int64_t pc = ((f->box_lo[l][2] + k) * pd.n[1] + f->box_lo[l][1] + j) * pd.n[0] + f->box_lo[l][0] + i;
                for (int v = 0; v < nv; ++v) {
                    double sum = 0.0;
                    for (int o = 0; o < nchild; ++o) {
                        int64_t ci = nd > 0 ? 2 * i + (o & 1) : i;
                        int64_t cj = nd > 1 ? 2 * j + ((o >> 1) & 1) : j;
                        int64_t ck = nd > 2 ? 2 * k + ((o >> 2) & 1) : k;
                        sum += Uchild[v * NC + (ck * cd.n[1] + cj) * cd.n[0] + ci];
                    }
                    Uparent[v * NP + pc] = sum / (double)nchild;
                }
            }
    return ORC_OK;
}

typedef struct {
    const orc_fmr_desc *f;
    orc_desc lev[ORC_FMR_MAXLEV];
    double *const *U;
    double *ext[ORC_FMR_MAXLEV];
    double T[ORC_FMR_MAXLEV];
    double *from_children[ORC_FMR_MAXLEV][3][2];
    double cfl, dt_fixed;
    int status;
} fmr_ctx;

/* number of faces normal to q of an (n0, n1, n2) block of cells: one per
 * transverse position */
static int64_t face_count(const int64_t n[3], int q) { return n[(q + 1) % 3] * n[(q + 2) % 3]; }

static void note(fmr_ctx *c, int st)
{
    if (st != ORC_OK && c->status == ORC_OK) c->status = st;
}

/* One two-stage step of level l with its exterior held in ext[l].
 * provisional: the first stage alone (the coarse level's provisional stage
 * between its child's two steps), no replacement.  acc, when given, accumulates the level's
 * own boundary fluxes integrated over the step (ForParents). */
static void level_step(fmr_ctx *c, int l, double dt, int provisional, double *acc[3][2])
{
    const orc_desc *d = &c->lev[l];
    int nd = d->ndim, nv = nvars(d);
    int64_t N = ncells(d), T = nv * N;
    double *U = c->U[l];
    const double *Uext = l > 0 ? c->ext[l] : NULL;
    double *L = (double *)malloc(sizeof(double) * T);
    if (provisional) {
        note(c, rhs_core(d, U, Uext, L, NULL));
        for (int64_t i = 0; i < T; ++i) U[i] = U[i] + dt * L[i];
        free(L);
        return;
    }
    int child = l + 1 < c->f->nlev;
    face_rec r[2];
    memset(r, 0, sizeof(r));
    int64_t cn[3] = {1, 1, 1};
    if (child)
        for (int q = 0; q < 3; ++q) cn[q] = c->f->box_n[l + 1][q];
    for (int s = 0; s < 2; ++s) {
        for (int q = 0; q < nd; ++q)
            for (int side = 0; side < 2; ++side) {
                if (acc) r[s].own[q][side] = (double *)malloc(sizeof(double) * nv * face_count(d->n, q));
                if (child) r[s].child[q][side] = (double *)malloc(sizeof(double) * nv * face_count(cn, q));
            }
        for (int q = 0; q < 3; ++q) {
            r[s].clo[q] = child ? c->f->box_lo[l + 1][q] : 0;
            r[s].cn[q] = cn[q];
        }
    }
    double *K1 = (double *)malloc(sizeof(double) * T);
    double *U1 = (double *)malloc(sizeof(double) * T);
    note(c, rhs_core(d, U, Uext, L, &r[0]));
    for (int64_t i = 0; i < T; ++i) {
        K1[i] = dt * L[i];
        U1[i] = U[i] + K1[i];
    }
    note(c, rhs_core(d, U1, Uext, L, &r[1]));
    for (int64_t i = 0; i < T; ++i) U[i] = U[i] + 0.5 * (K1[i] + dt * L[i]);

    if (child && !c->f->no_reflux) {
        for (int q = 0; q < nd; ++q) {
            int r1 = (q + 1) % 3, r2 = (q + 2) % 3;
            double dq = cell_width(d, q);
            int64_t nf = face_count(cn, q);
            for (int side = 0; side < 2; ++side)
                for (int64_t t2 = 0; t2 < cn[r2]; ++t2)
                    for (int64_t t1 = 0; t1 < cn[r1]; ++t1) {
                        int64_t t = t2 * cn[r1] + t1, x[3];
                        x[q] = side == 0 ? r[0].clo[q] - 1 : r[0].clo[q] + cn[q];
                        x[r1] = r[0].clo[r1] + t1;
                        x[r2] = r[0].clo[r2] + t2;
                        int64_t cell = (x[2] * d->n[1] + x[1]) * d->n[0] + x[0];
                        for (int v = 0; v < nv; ++v) {
                            double phi_c = 0.5 * dt * (r[0].child[q][side][v * nf + t] + r[1].child[q][side][v * nf + t]);
                            double phi_f = c->from_children[l][q][side][v * nf + t];
                            double corr = side == 0 ? phi_c - phi_f : phi_f - phi_c;
                            U[v * N + cell] += corr / dq;
                        }
                    }
        }
    }
    if (acc)
        for (int q = 0; q < nd; ++q)
            for (int side = 0; side < 2; ++side) {
                int64_t m = nv * face_count(d->n, q);
                for (int64_t i = 0; i < m; ++i)
                    acc[q][side][i] += 0.5 * dt * (r[0].own[q][side][i] + r[1].own[q][side][i]);
            }
    for (int s = 0; s < 2; ++s)
        for (int q = 0; q < 3; ++q)
            for (int side = 0; side < 2; ++side) {
                free(r[s].own[q][side]);
                free(r[s].child[q][side]);
            }
    free(K1);
    free(U1);
    free(L);
}

/* The coarse level's share of its child's two steps: the child's boundary
 * fluxes accumulated over them (acc, on the child's faces) restricted to
 * this level's faces of the child box, each coarse face the mean of its
 * 2^(d-1) fine faces. */
static void restrict_boundary_fluxes(fmr_ctx *c, int l, double *const acc[3][2])
{
    const orc_fmr_desc *f = c->f;
    const orc_desc *cd = &c->lev[l + 1];
    int nv = nvars(&f->base), nd = f->base.ndim;
    int64_t cn[3] = {f->box_n[l + 1][0], f->box_n[l + 1][1], f->box_n[l + 1][2]};
    for (int q = 0; q < nd; ++q) {
        int r1 = (q + 1) % 3, r2 = (q + 2) % 3;
        int64_t nf = face_count(cn, q), nff = face_count(cd->n, q);
        int a1 = r1 < nd ? 2 : 1, a2 = r2 < nd ? 2 : 1;
        for (int s = 0; s < 2; ++s)
            for (int v = 0; v < nv; ++v)
                for (int64_t t2 = 0; t2 < cn[r2]; ++t2)
                    for (int64_t t1 = 0; t1 < cn[r1]; ++t1) {
                        double sum = 0.0;
                        for (int o2 = 0; o2 < a2; ++o2)
                            for (int o1 = 0; o1 < a1; ++o1)
                                sum += acc[q][s][v * nff + (a2 * t2 + o2) * cd->n[r1] + a1 * t1 + o1];
                        c->from_children[l][q][s][v * nf + t2 * cn[r1] + t1] = sum / (double)(a1 * a2);
                    }
    }
}

/* One global step of the nested levels (Sec. 3.6, Algs. Evolve, EvolveLevel
 * and StepLevel), written as the time-ordered schedule those algorithms
 * produce.  Level l takes two steps for each step of level l - 1, so the
 * deepest level D takes 2^D steps; its step is the CFL step, and each
 * coarser level's step spans its child's two steps, so a coarse level steps
 * only after its child has.  Between the child's first and second step the
 * coarse level takes a provisional first stage over the child's first step
 * (from a saved copy of its state, restored afterwards), so that the child's
 * exterior for its second step is prolonged from the coarse state at the
 * child's time.  A full coarse step replaces the fluxes through the child
 * box's faces by the child's (their time integral over its two steps) and is
 * followed by the restriction of the child onto the cells it covers.  In
 * schedule terms: after the deepest step k, level l (from D - 1 up) has just
 * seen its child finish that child's step number m = (k + 1) / 2^(D-1-l); an
 * odd m (a first step) calls for the provisional stage of level l and ends
 * the cascade, an even m for the full step of level l, after which its own
 * parent is looked at. */
int orc_fmr_step(const orc_fmr_desc *f, double *const *U, double cfl, double dt_fixed, double *dt_out)
{
    if (!fmr_valid(f) || !U || !dt_out) return ORC_EINVAL;
    if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return ORC_EINVAL;
    fmr_ctx c;
    memset(&c, 0, sizeof(c));
    c.f = f;
    c.U = U;
    c.cfl = cfl;
    c.dt_fixed = dt_fixed;
    int nv = nvars(&f->base), nd = f->base.ndim;
    /* own[l]: level l's boundary fluxes accumulated over its parent's
     * current step; saved[l]: level l's state during its provisional stage */
    double *own[ORC_FMR_MAXLEV][3][2];
    double *saved[ORC_FMR_MAXLEV];
    memset(own, 0, sizeof(own));
    memset(saved, 0, sizeof(saved));
    for (int l = 0; l < f->nlev; ++l) {
        orc_fmr_level(f, l, &c.lev[l]);
        if (l > 0) {
            ghost_geom G = make_geom(&c.lev[l]);
            c.ext[l] = (double *)calloc((size_t)(nv * G.m[0] * G.m[1] * G.m[2]), sizeof(double));
            for (int q = 0; q < nd; ++q)
                for (int s = 0; s < 2; ++s)
                    own[l][q][s] = (double *)calloc((size_t)(nv * face_count(c.lev[l].n, q)), sizeof(double));
        }
        if (l + 1 < f->nlev) {
            for (int q = 0; q < nd; ++q)
                for (int s = 0; s < 2; ++s)
                    c.from_children[l][q][s] =
                        (double *)calloc((size_t)(nv * face_count(f->box_n[l + 1], q)), sizeof(double));
            saved[l] = (double *)malloc(sizeof(double) * (size_t)(nv * ncells(&c.lev[l])));
        }
    }
    const int D = f->nlev - 1;
    const long nsteps = 1L << D;
    for (long k = 0; k < nsteps && c.status == ORC_OK; ++k) {
        /* the deepest level's step: exterior from its parent, CFL step */
        double dt;
        if (D > 0) note(&c, orc_fmr_prolong(f, D, c.U[D - 1], c.ext[D]));
        if (c.dt_fixed > 0.0) dt = c.dt_fixed;
        else note(&c, orc_cfl_dt(&c.lev[D], c.U[D], c.cfl, &dt));
        level_step(&c, D, dt, 0, D > 0 ? own[D] : NULL);
        c.T[D] += dt;
        for (int l = D - 1; l >= 0; --l) {
            const long m = (k + 1) >> (D - 1 - l);
            const int64_t T = nv * ncells(&c.lev[l]);
            if (m & 1) {
                /* the child's first step is done: the provisional stage */
                memcpy(saved[l], c.U[l], sizeof(double) * (size_t)T);
                if (l > 0) note(&c, orc_fmr_prolong(f, l, c.U[l - 1], c.ext[l]));
                level_step(&c, l, c.T[l + 1] - c.T[l], 1, NULL);
                break;
            }
            /* both child steps are done: the full step of level l */
            memcpy(c.U[l], saved[l], sizeof(double) * (size_t)T);
            restrict_boundary_fluxes(&c, l, own[l + 1]);
            for (int q = 0; q < nd; ++q)
                for (int s = 0; s < 2; ++s)
                    memset(own[l + 1][q][s], 0, sizeof(double) * (size_t)(nv * face_count(c.lev[l + 1].n, q)));
            if (l > 0) note(&c, orc_fmr_prolong(f, l, c.U[l - 1], c.ext[l]));
            dt = c.T[l + 1] - c.T[l];
            level_step(&c, l, dt, 0, l > 0 ? own[l] : NULL);
            note(&c, orc_fmr_restrict(f, l + 1, c.U[l + 1], c.U[l]));
            c.T[l] += dt;
        }
    }
    for (int l = 1; l < f->nlev; ++l)
        if (c.T[l] != c.T[0]) note(&c, ORC_EINVAL);
    *dt_out = c.T[0];
    for (int l = 0; l < f->nlev; ++l) {
        free(c.ext[l]);
        free(saved[l]);
        for (int q = 0; q < 3; ++q)
            for (int s = 0; s < 2; ++s) {
                free(c.from_children[l][q][s]);
                free(own[l][q][s]);
            }
    }
    return c.status;
}
