// stage.hip -- one Runge-Kutta stage of the finite-volume update, fused into
// a single gfx950 kernel.
//
// Per cell the kernel performs, in the paper's order (Sec. 3, Alg. 1):
// primitive recovery (Sec. 3.5), ghost values by index mapping (the boundary
// step), generalised-minmod slopes (eq. MinMod) or learned slopes, face states
// (eqs. conservedLeft..conservedRight), the HLL or HLLC flux (eqs. FluxHLL,
// FluxHLLC with eq. MiddleWaveSpeed and the middle states), the flux
// divergence plus a uniform-gravity source (eq. BalanceEquationAverage), and
// the Runge-Kutta combination (eqs. RungeKutta1-3, written as
// U^(1) = U^n + dt L(U^n) and U^{n+1} = (U^n + U^(1) + dt L(U^(1))) / 2).
// The second stage also reduces the CFL rate (eq. courantTimeStep) of the
// state it writes.
//
// Layout: SoA state arrays, one per conserved variable, x fastest, interior
// cells only.  Tiling: a block owns a 64 x BY column tile of the x-y plane and
// marches along z.  The z stencil lives in registers (a 3-plane window of
// primitives plus the carried z-face flux), so every z face is solved once and
// no z halo is re-read.  The current x-y plane, with a 2-cell halo, is staged
// in LDS; slopes and face fluxes go through LDS so every x and y face is also
// solved once.  Ghost cells are never stored: out-of-range indices are mapped
// to their interior source (periodic wrap, outflow clamp, reflecting mirror
// with the normal velocity negated).
#include "hy_internal.h"
#include "hy_face.h"
#include "hy_ride.h"

#include <math.h>
#include <type_traits>

namespace hy {
namespace {

// ------------------------------------------------------------ kernel ----

template <int ND, typename T>
__device__ __forceinline__ double stage_dt(const StageArgs<T> &a)
{
    if (a.dt_mode == DT_HOST) return a.dt_host;
    if (a.dt_mode == DT_PTR) return *a.dt_dev;
    unsigned long long rb = 0ull;
#pragma unroll
    for (int k = 0; k < RATE_SLOTS; ++k) rb = rb > a.ctl->rate[a.parity][k] ? rb : a.ctl->rate[a.parity][k];
    const double rate = __longlong_as_double((long long)rb);
    const double t = a.ctl->time[a.parity];
    double dt = fmin(a.cfl / rate, a.t_end - t);
    return dt > 0.0 ? dt : 0.0;
}

// A value every lane holds alike, moved to a scalar register so the vector
// register budget of the per-cell work does not carry it.
__device__ __forceinline__ float uniform_(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uniform_(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

constexpr int FLIP = 1 << 30;      // set on a mapped index whose source is a mirror image
constexpr int IDX = FLIP - 1;

// Source of index i along a dimension of n interior cells; flip toggles when
// the source is a mirror image.  Indices far outside the ghost range (only
// met by the unused columns of partial tiles) are clamped into the array.
__device__ __forceinline__ int map32(int i, int n, int bclo, int bchi, bool &flip)
{
    if (i >= 0 && i < n) return i;
    int m;
    if (i < 0) {
        if (bclo == BC_PERIODIC) m = i + n;
        else if (bclo == BC_OUTFLOW) m = 0;
        else { m = -1 - i; flip = !flip; }
    } else {
        if (bchi == BC_PERIODIC) m = i - n;
        else if (bchi == BC_OUTFLOW) m = n - 1;
        else { m = 2 * n - 1 - i; flip = !flip; }
    }
    return m < 0 ? 0 : (m >= n ? n - 1 : m);
}

// The learned-limiter slope of variable v along q at cell (gx, gy, gz) (face
// values w +/- slope / 2): interior slopes come from the slope array; a ghost
// cell along q takes the slope of its interior source (periodic), zero
// (outflow) or the mirrored slope (reflecting; the normal velocity is odd, the
// other variables even)
template <int ND, typename T>
__device__ __forceinline__ T learned_slope(const StageArgs<T> &a, int q, int v, int gx, int gy, int gz)
{
    int g[3] = {gx, gy, gz};
    T sgn = T(1);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        if (r >= ND) { g[r] = 0; continue; }
        const int n = (int)a.n[r];
        int i = g[r];
        if (i >= 0 && i < n) continue;
        if (r == q) {
            const int bc = i < 0 ? a.bc[r][0] : a.bc[r][1];
            if (bc == BC_OUTFLOW) return T(0);
            if (bc == BC_PERIODIC) i = i < 0 ? i + n : i - n;
            else { i = i < 0 ? -1 - i : 2 * n - 1 - i; sgn = (v == 1 + q) ? T(1) : T(-1); }
        }
        g[r] = i < 0 ? 0 : (i >= n ? n - 1 : i);
    }
    const int c = (g[2] * (int)a.n[1] + g[1]) * (int)a.n[0] + g[0];
    const float *base = a.slopes + (int64_t)(q * (ND + 2) + v) * a.vstride;
    return sgn * (T)base[c];
}

// The face-flux workgroups of a padded launch (see BoxFluxes): workgroup fid
// after the tiles takes (box, q, side) = segment fid / blocks, NT faces of it.
template <int ND, int SOLVER, int NT, typename T>
__device__ __forceinline__ void stage_box_faces(const StageArgs<T> &a, int fid, int tid)
{
    const int seg = fid / a.bf.blocks;
    const int t = (fid - seg * a.bf.blocks) * NT + tid;
    const int side = seg & 1, bq = seg >> 1, k = bq / ND, q = bq - k * ND;
    const Grid g{{a.vm[0], a.vm[1], a.vm[2]}, a.vstride};
    const Box &b = a.bf.b[k];
    const double w = 0.5 * *a.dt_dev;
    const bool as = a.bf.assign[k] != 0;
    if (q == 0)
        box_faces<ND, 0, SOLVER>(a.uin, g, b, t, side, a.gamma, a.gm1, a.inv_gm1, a.theta, w, as, a.bf.acc[k][0][0],
                                 a.bf.acc[k][0][1]);
    if constexpr (ND >= 2)
        if (q == 1)
            box_faces<ND, 1, SOLVER>(a.uin, g, b, t, side, a.gamma, a.gm1, a.inv_gm1, a.theta, w, as,
                                     a.bf.acc[k][1][0], a.bf.acc[k][1][1]);
    if constexpr (ND >= 3)
        if (q == 2)
            box_faces<ND, 2, SOLVER>(a.uin, g, b, t, side, a.gamma, a.gm1, a.inv_gm1, a.theta, w, as,
                                     a.bf.acc[k][2][0], a.bf.acc[k][2][1]);
}

// At least 4 waves per SIMD: the LDS plane tile admits two 512-thread
// workgroups per CU, so registers beyond 128 per lane would only cost occupancy.
template <int ND, typename T, int SOLVER, int STAGE, int LIM, int BX, int BY>
// 512-thread tiles: four waves per SIMD (two workgroups per CU); 256-thread
// tiles: three, which leaves the 3D kernels room to prefetch without spilling
// (their LDS would allow four workgroups, but the registers then spill)
__global__ void __launch_bounds__(BX *BY, (BX * BY == 256) ? 3 : 4) k_stage(const StageArgs<T> a)
{
    constexpr int NP = ND + 2;
    constexpr int IP = ND + 1;
    constexpr int NT = BX * BY;
    static_assert(NT % 64 == 0, "plane tiles are whole wavefronts");
    constexpr int RY = (ND >= 2) ? BY + 4 : 1;  // LDS rows of primitives (2-cell halo in y)
    constexpr int OY = (ND >= 2) ? 2 : 0;       // row offset of the tile in LDS
    constexpr int WX = BX + 4;                  // LDS columns (2-cell halo in x)
    constexpr int SYR = (ND >= 2) ? BY + 2 : 1;
    constexpr int FYR = (ND >= 2) ? BY + 1 : 1;
    constexpr int HROW = (ND >= 2) ? 4 * WX : 0;  // halo rows -2, -1, BY, BY+1 (full width)
    constexpr int NH = HROW + 4 * BY;             // + halo columns -2, -1, BX, BX+1 of each tile row
    constexpr int HPT = (NH + NT - 1) / NT;       // halo cells per thread

    __shared__ T sW[NP][RY][WX];        // primitives of the current plane
    __shared__ T sSx[NP][BY][BX + 2];   // x slopes of cells -1 .. BX
    __shared__ T sSy[NP][SYR][BX];      // y slopes of rows -1 .. BY
    __shared__ T sFx[NP][BY][BX + 1];   // x faces 0 .. BX (face f between cells f-1, f)
    __shared__ T sFy[NP][FYR][BX];      // y faces 0 .. BY
    __shared__ int sMap[WX + RY];       // mapped x of columns -2 .. BX+1, then mapped y of rows -2 .. BY+1
    // HLLC switch: the shock-detector bits of the current plane (cells of
    // rows -1 .. BY and columns -1 .. BX, corners unused), and in 3D the
    // pressure and in-plane velocities of the next plane over the same cells
    constexpr bool SW = SOLVER == SOLVER_HLLC_SWITCH;
    constexpr bool SW3 = SW && ND == 3;
    __shared__ uint8_t sB[SW ? BY + 2 : 1][SW ? BX + 2 : 1];
    __shared__ T sN[SW3 ? 3 : 1][SW3 ? BY + 2 : 1][SW3 ? BX + 2 : 1];
    // (3D switch) p and v_z of the plane below the current one, own and ring
    // cells: each thread reads and rewrites only its own cells' entries
    __shared__ T sC[SW3 ? 2 : 1][SW3 ? BY + 2 : 1][SW3 ? BX + 2 : 1];
    // (3D switch) v_z of the ring cells in the next plane (p sits in sN)
    __shared__ T sV[SW3 ? BY + 2 : 1][SW3 ? BX + 2 : 1];

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * BX + tx;
    const int nx = (int)a.n[0], ny = (int)a.n[1], nz = (int)a.n[2];
    // storage: interior cells only, or (a view of a padded array) the n cells
    // from storage cell voff of an array of extents vm, with the 2 cells
    // around them read as ghosts
    constexpr bool PAD = LIM == LIM_THETA_PADDED;
    static_assert(!PAD || SOLVER != SOLVER_HLLC_SWITCH, "padded arrays take HLL or HLLC");
    if constexpr (PAD) {
        // the workgroups after the tiles compute box face fluxes, then those
        // after them run the job riding on the launch (whole workgroups,
        // before any barrier)
        if ((int)blockIdx.x >= a.ntiles) {
            const int fid = (int)blockIdx.x - a.ntiles;
            if (fid < a.nbfwg) stage_box_faces<ND, SOLVER, NT>(a, fid, tid);
            else ride_run<ND>(a.ride, fid - a.nbfwg, tid, NT);
            return;
        }
    }
    const int vx = PAD ? a.voff[0] : 0, vy = (PAD && ND >= 2) ? a.voff[1] : 0, vz = (PAD && ND == 3) ? a.voff[2] : 0;
    const int sx = PAD ? a.vm[0] : nx;
    const int plane = PAD ? a.vm[0] * a.vm[1] : nx * ny;
    // a coordinate's storage index: boundary-mapped, or (a view) shifted by
    // the view offset and clamped to the ghost layers (the unused columns of
    // partial tiles)
    auto smap = [&](int i, int n, int off, int bclo, int bchi, bool &f) -> int {
        if constexpr (PAD) return (i < -2 ? -2 : (i > n + 1 ? n + 1 : i)) + off;
        return map32(i, n, bclo, bchi, f);
    };
    // XCD-aware tile order: consecutive workgroup ids are dealt round-robin
    // to the 8 XCDs, so hand each XCD a contiguous band of tiles (x fastest,
    // then y, then z chunk); neighbouring tiles then share halo lines in the
    // same L2.  The mapping is a bijection whatever the dispatch order.
    int bxi, byi, bzi;
    {
        const int lid = blockIdx.x, total = a.ntiles;
        const int per = total >> 3, rem = total & 7, xcd = lid & 7;
        const int logical = xcd * per + (xcd < rem ? xcd : rem) + (lid >> 3);
        bxi = logical % a.tiles_x;
        const int rest = logical / a.tiles_x;
        byi = rest % a.tiles_y;
        bzi = rest / a.tiles_y;
    }
    const int x0 = bxi * BX;
    const int y0 = (ND >= 2) ? byi * BY : 0;
    const int z0 = (ND == 3) ? bzi * a.zchunk : 0;
    const int nplanes = (ND == 3) ? (z0 + a.zchunk <= nz ? a.zchunk : nz - z0) : 1;
    const T gamma = a.gamma, gm1 = a.gm1, igm1 = a.inv_gm1;
    const T sg = uniform_(sqrt_gamma(gamma));
    // face value = w +/- hs * slope: the minmod path keeps the slope divided
    // by theta (slope_mm), the learned path the slope itself
    const ThetaLim<T> tl = theta_lim(a.theta);
    const T lk = uniform_(tl.k);
    const T hs = LIM == LIM_LEARNED ? T(0.5) : uniform_(tl.hs);
    const bool grav = a.accel[0] != T(0) || a.accel[1] != T(0) || a.accel[2] != T(0);  // uniform

    // per-variable base pointers (uniform), 32-bit cell offsets below
    const T *uin[NP];
    const T *u0p[NP];
    T *uout[NP];
#pragma unroll
    for (int v = 0; v < NP; ++v) {
        uin[v] = a.uin + (int64_t)v * a.vstride;
        u0p[v] = a.u0 + (int64_t)v * a.vstride;
        uout[v] = a.uout + (int64_t)v * a.vstride;
    }
    // cell offsets are < 2^32 / sizeof(T) (checked on the host), so byte
    // offsets stay 32-bit and loads use the scalar-base + vector-offset form
    auto at = [](const T *base, unsigned off) -> const T & {
        return *(const T *)((const char *)base + off * (unsigned)sizeof(T));
    };
    auto load = [&](unsigned off, T (&u)[NP]) {
#pragma unroll
        for (int v = 0; v < NP; ++v) u[v] = at(uin[v], off);
    };

    for (int i = tid; i < WX + RY; i += NT) {
        bool f = false;
        int m = 0;
        if (i < WX) m = smap(x0 + i - 2, nx, vx, a.bc[0][0], a.bc[0][1], f);
        else if (ND >= 2) m = smap(y0 + (i - WX) - 2, ny, vy, a.bc[1][0], a.bc[1][1], f);
        sMap[i] = m | (f ? FLIP : 0);
    }

    const double dtd = stage_dt<ND>(a);
    const T dt = (T)dtd;
    // the step's weight of a flux difference per unit width, and of the source
    const T wdt = STAGE == 1 ? dt : T(0.5) * dt;
    T cdt[3], cacc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        cdt[d] = uniform_(wdt * a.idx[d]);
        cacc[d] = uniform_(wdt * a.accel[d]);
    }
    if constexpr (STAGE == 1) {
        if (blockIdx.x == 0 && tid < RATE_SLOTS) {
            a.ctl->rate[a.parity ^ 1][tid] = 0ull;
            if (tid == 0) a.ctl->time[a.parity ^ 1] = a.ctl->time[a.parity] + dtd;
        }
    }
    __syncthreads();

    // own column: mapped (the unused columns of partial tiles hold ghost values)
    const int xm = sMap[tx + 2];
    const int ym = (ND >= 2) ? sMap[WX + ty + 2] : 0;
    const bool fxo = (xm & FLIP) != 0, fyo = (ym & FLIP) != 0;
    const unsigned colo = (unsigned)((ym & IDX) * sx + (xm & IDX));
    const int gx = x0 + tx, gy = y0 + ty;
    const bool own_valid = (gx < nx) && (gy < ny);
    const unsigned colv = (unsigned)((gy + vy) * sx + gx + vx);

    // halo cells of this thread: plane offset, LDS slot, mirror flags
    unsigned hoff[HPT];
    int hlds[HPT], hflg[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const int h = tid + j * NT;
        hlds[j] = -1;
        hoff[j] = 0;
        hflg[j] = 0;
        if (h < NH) {
            int row, col;
            if (h < HROW) {
                const int hr = h / WX;
                row = hr < 2 ? hr - 2 : BY + hr - 2;
                col = h - hr * WX - 2;
            } else {
                const int jj = h - HROW;
                row = jj >> 2;
                const int cc = jj & 3;
                col = cc < 2 ? cc - 2 : BX + cc - 2;
            }
            const int hx = sMap[col + 2];
            const int hy = (ND >= 2) ? sMap[WX + row + 2] : 0;
            hoff[j] = (unsigned)((hy & IDX) * sx + (hx & IDX));
            hlds[j] = (row + OY) * WX + col + 2;
            hflg[j] = ((hx & FLIP) ? 1 : 0) | ((hy & FLIP) ? 2 : 0);
        }
    }

    // HLLC switch, detector of Sec. 3.2's switch (the reading the oracle
    // takes): a cell is in a shock moving along q when the pressures of its
    // neighbours along q differ by more than eps times the smaller one and
    // the velocity along q decreases across it; a face normal to r takes HLL
    // when one of its two cells is flagged along some q != r.  Ring item rt
    // (rows -1 and BY of the tile, then columns -1 and BX of its rows) goes to
    // thread RING0 + rt: whole wavefronts after the first 2 BX threads, which
    // carry the y-ring slopes, so the ring work of the two does not pile up on
    // the same wavefronts; its ghost values come through the same boundary
    // map (and mirror signs) as the halo.
    constexpr int NRING = 2 * BX + 2 * BY;
    constexpr int RING0 = ((NT - NRING < 2 * BX ? NT - NRING : 2 * BX) / 64) * 64;
    static_assert(!SW || (RING0 >= 0 && RING0 + NRING <= NT), "ring items fit the workgroup");
    const int rt = tid - RING0;
    const bool ringt = SW && rt >= 0 && rt < NRING;
    // the ring cell's tile row and column (formed where used, so nothing of
    // it stays in registers through the march)
    auto ring_rc = [&](int &r, int &c) {
        if (rt < 2 * BX) {
            r = rt < BX ? -1 : BY;
            c = rt < BX ? rt : rt - BX;
        } else {
            const int e = rt - 2 * BX;
            r = e >> 1;
            c = (e & 1) ? BX : -1;
        }
    };
    const T seps = (T)SHOCK_EPS;
    auto shock = [&](T pa, T pb, T va, T vb) -> bool {
        return (fabs(pb - pa) > seps * fmin(pa, pb)) & (vb - va < T(0));
    };
    // x and y bits of the cell at tile (row r, column c) of the current plane
    auto bits_w = [&](int r, int c) -> unsigned {
        unsigned b = shock(sW[IP][r + OY][c + 1], sW[IP][r + OY][c + 3], sW[1][r + OY][c + 1], sW[1][r + OY][c + 3]);
        if constexpr (ND >= 2)
            b |= shock(sW[IP][r + OY - 1][c + 2], sW[IP][r + OY + 1][c + 2], sW[2][r + OY - 1][c + 2],
                       sW[2][r + OY + 1][c + 2])
                 << 1;
        return b;
    };
    // x and y bits of the own cell in the plane held by sN
    auto bits_n = [&]() -> unsigned {
        if constexpr (SW3) {
            return (unsigned)shock(sN[0][ty + 1][tx], sN[0][ty + 1][tx + 2], sN[1][ty + 1][tx], sN[1][ty + 1][tx + 2]) |
                   ((unsigned)shock(sN[0][ty][tx + 1], sN[0][ty + 2][tx + 1], sN[2][ty][tx + 1], sN[2][ty + 2][tx + 1])
                    << 1);
        }
        return 0u;
    };

    bool bad = false;
    T rate = T(0);
    // (uniform) mirror images only where a face reflects, and the CFL rate
    // as (max_q |v_q| + c) / dq when the cells are cubes (the same value:
    // (x + c) / dq rounds monotonically in x)
    bool mir = false;
#pragma unroll
    for (int q = 0; q < ND; ++q) mir |= (a.bc[q][0] == BC_REFLECT) | (a.bc[q][1] == BC_REFLECT);
    const bool cubic = (ND < 2 || a.idx[1] == a.idx[0]) && (ND < 3 || a.idx[2] == a.idx[0]);

    auto to_w = [&](const T (&u)[NP], T (&w)[NP], bool fx, bool fy, bool fz) {
        bad |= !to_prim<ND>(u, w, gm1);
        if (fx) w[1] = -w[1];
        if constexpr (ND >= 2) { if (fy) w[2] = -w[2]; }
        if constexpr (ND == 3) { if (fz) w[3] = -w[3]; }
    };
    auto zoff = [&](int z, bool &fz) -> unsigned {
        if constexpr (ND == 3) return (unsigned)(smap(z, nz, vz, a.bc[2][0], a.bc[2][1], fz) * plane);
        return 0u;
    };
    auto face_state = [&](const T (&w)[NP], const T (&s)[NP], T h, T (&out)[NP]) {
#pragma unroll
        for (int v = 0; v < NP; ++v) out[v] = w[v] + h * s[v];
    };
    // the ring cell of this thread at plane z: pressure and the three
    // velocities, mirror signs applied (3D switch)
    auto ring_prim = [&](int z, int r, int c, T &p, T &vxr, T &vyr, T &vzr) {
        bool fz = false;
        T u[NP], w[NP];
        const int rmx = sMap[c + 2], rmy = sMap[WX + r + 2];
        load(zoff(z, fz) + (unsigned)((rmy & IDX) * sx + (rmx & IDX)), u);
        (void)to_prim<ND>(u, w, gm1);
        p = w[IP];
        vxr = (rmx & FLIP) ? -w[1] : w[1];
        vyr = (rmy & FLIP) ? -w[2] : w[2];
        vzr = fz ? -w[3] : w[3];
    };

    // register z window: W (primitives), U (conserved), S (z slopes) and F
    // (z face fluxes) of three consecutive planes, rotated by renaming
    T WA[NP], WB[NP], WC[NP], UA[NP], UB[NP], UC[NP], SA[NP], SB[NP], SC[NP], FA[NP], FB[NP], FC[NP];
    if constexpr (ND == 3) {
        T um[NP], wm2[NP], wm1[NP], sm1[NP];
        bool f2 = false, f1 = false, f0 = false, fp = false;
        load(zoff(z0 - 2, f2) + colo, um);
        to_w(um, wm2, fxo, fyo, f2);
        load(zoff(z0 - 1, f1) + colo, um);
        to_w(um, wm1, fxo, fyo, f1);
        load(zoff(z0, f0) + colo, UA);
        to_w(UA, WA, fxo, fyo, f0);
        load(zoff(z0 + 1, fp) + colo, UB);
        to_w(UB, WB, fxo, fyo, fp);
#pragma unroll
        for (int v = 0; v < NP; ++v) {
            if constexpr (LIM != LIM_LEARNED) {
                sm1[v] = slope_mm(wm2[v], wm1[v], WA[v], lk);
                SA[v] = slope_mm(wm1[v], WA[v], WB[v], lk);
            } else {
                sm1[v] = learned_slope<ND>(a, 2, v, gx, gy, z0 - 1);
                SA[v] = learned_slope<ND>(a, 2, v, gx, gy, z0);
            }
        }
        T fl[NP], fr[NP];
        face_state(wm1, sm1, hs, fl);
        face_state(WA, SA, -hs, fr);
        bool hll = false;
        if constexpr (SW3) {
            // the face below the chunk: x and y bits of planes z0 - 1 and z0
            // (their in-plane neighbours through sN, one plane at a time)
            T p, vxr, vyr, vzr;
            int rr = 0, rc = 0;
            ring_rc(rr, rc);
            sN[0][ty + 1][tx + 1] = wm1[IP];
            sN[1][ty + 1][tx + 1] = wm1[1];
            sN[2][ty + 1][tx + 1] = wm1[2];
            if (ringt) {
                ring_prim(z0 - 1, rr, rc, p, vxr, vyr, vzr);
                sN[0][rr + 1][rc + 1] = p;
                sN[1][rr + 1][rc + 1] = vxr;
                sN[2][rr + 1][rc + 1] = vyr;
                sC[0][rr + 1][rc + 1] = p;
                sC[1][rr + 1][rc + 1] = vzr;
            }
            sC[0][ty + 1][tx + 1] = wm1[IP];
            sC[1][ty + 1][tx + 1] = wm1[3];
            __syncthreads();
            const unsigned xym = bits_n();
            __syncthreads();
            sN[0][ty + 1][tx + 1] = WA[IP];
            sN[1][ty + 1][tx + 1] = WA[1];
            sN[2][ty + 1][tx + 1] = WA[2];
            if (ringt) {
                ring_prim(z0, rr, rc, p, vxr, vyr, vzr);
                sN[0][rr + 1][rc + 1] = p;
                sN[1][rr + 1][rc + 1] = vxr;
                sN[2][rr + 1][rc + 1] = vyr;
            }
            __syncthreads();
            hll = (xym | bits_n()) != 0u;
            __syncthreads();
        }
        face_flux<ND, 2, SOLVER>(fl, fr, FA, sg, igm1, hll);
    } else {
        load(colo, UA);
        to_w(UA, WA, fxo, fyo, false);
    }

    // halo cells of the next plane, loaded one plane ahead so their latency
    // is not on the path to the first barrier of the plane
    T hnext[HPT][NP];
    auto load_halo = [&](int z, T (&h)[HPT][NP]) {
        const unsigned zo = (ND == 3) ? (unsigned)(((z < nz ? z : nz - 1) + vz) * plane) : 0u;
#pragma unroll
        for (int j = 0; j < HPT; ++j)
            if (hlds[j] >= 0) load(zo + hoff[j], h[j]);
    };
    // (the learned-limiter kernels hold the prefetched slopes and the switch
    // kernels the detector's state; to stay within the register budget of
    // four waves per SIMD they load the halo and the second stage's U^n when
    // they are used instead of ahead.  The switch's 256-thread tiles run at
    // three waves per SIMD, which leaves them room for both prefetches)
    constexpr bool LATE = (SW && NT == 512) || LIM == LIM_LEARNED;
    if constexpr (!LATE) load_halo(z0, hnext);

    T *sWf = &sW[0][0][0];
    // one plane: Wk/Uk/Sk/Flo hold plane kz, Wk1/Uk1 plane kz+1; the body
    // fills W2/U2 (plane kz+2), Sk1 (z slopes of kz+1) and Fhi (face kz+1/2)
    auto body = [&](int it, T (&Wk)[NP], T (&Wk1)[NP], T (&W2)[NP], T (&Uk)[NP], T (&Uk1)[NP], T (&U2)[NP],
                    T (&Sk)[NP], T (&Sk1)[NP], T (&Flo)[NP], T (&Fhi)[NP]) {
        (void)Uk1;
        const int kz = z0 + it;
        const unsigned zko = (ND == 3) ? (unsigned)((kz + vz) * plane) : 0u;
        bool fz2 = false;
        if constexpr (ND == 3) load(zoff(kz + 2, fz2) + colo, U2);
        T u0[NP];  // U^n of the own cell (second stage), issued early, used in phase 3
        if constexpr (STAGE == 2 && !LATE) {
#pragma unroll
            for (int v = 0; v < NP; ++v) u0[v] = own_valid ? at(u0p[v], zko + colv) : T(0);
        }

        // learned limiter: the own cell's x and y slopes and this thread's
        // ring slope go from the slope array straight into the LDS slope
        // tiles (free until phase 2) before the first barrier, so none of
        // them is held in registers across it; the z slope of plane kz+1 is
        // loaded in phase 1, where it is used
        T lsx[NP], lsy[NP], lry[NP], lrx[NP];
        const int ering = tid - (NT - 2 * BY);  // x ring item of the last threads
        if constexpr (LIM == LIM_LEARNED) {
            if (own_valid) {
                // an interior cell: the slopes sit at its own offset
                const unsigned o = zko + colv;
#pragma unroll
                for (int v = 0; v < NP; ++v) {
                    lsx[v] = (T)at(a.slopes + (int64_t)v * a.vstride, o);
                    if constexpr (ND >= 2) lsy[v] = (T)at(a.slopes + (int64_t)(NP + v) * a.vstride, o);
                }
            } else {  // a ghost column of a partial tile: boundary-mapped slopes
#pragma unroll
                for (int v = 0; v < NP; ++v) {
                    lsx[v] = learned_slope<ND>(a, 0, v, gx, gy, kz);
                    if constexpr (ND >= 2) lsy[v] = learned_slope<ND>(a, 1, v, gx, gy, kz);
                }
            }
#pragma unroll
            for (int v = 0; v < NP; ++v) {
                sSx[v][ty][tx + 1] = lsx[v];
                if constexpr (ND >= 2) sSy[v][ty + 1][tx] = lsy[v];
            }
            // ring slope of cell (rx, ry): direct inside the domain, boundary
            // mapped for a ghost (in 3D the extra code path costs more
            // registers than the index arithmetic it saves: measured)
            auto ring_slope = [&](int q, int rx, int ry, T (&out)[NP]) {
                if (ND < 3 && rx >= 0 && rx < nx && ry >= 0 && ry < ny) {
                    const unsigned o = zko + (unsigned)(ry * nx + rx);
#pragma unroll
                    for (int v = 0; v < NP; ++v) out[v] = (T)at(a.slopes + (int64_t)(q * NP + v) * a.vstride, o);
                } else {
#pragma unroll
                    for (int v = 0; v < NP; ++v) out[v] = learned_slope<ND>(a, q, v, rx, ry, kz);
                }
            };
            if constexpr (ND >= 2) {
                if (tid < 2 * BX) {
                    ring_slope(1, x0 + (tid < BX ? tid : tid - BX), y0 + (tid < BX ? -1 : BY), lry);
#pragma unroll
                    for (int v = 0; v < NP; ++v) sSy[v][tid < BX ? 0 : BY + 1][tid < BX ? tid : tid - BX] = lry[v];
                }
            }
            if (ering >= 0) {
                ring_slope(0, x0 + ((ering & 1) ? BX : -1), y0 + (ering >> 1), lrx);
#pragma unroll
                for (int v = 0; v < NP; ++v) sSx[v][ering >> 1][(ering & 1) ? BX + 1 : 0] = lrx[v];
            }
        }

        // ---- phase 0: primitives of plane kz into LDS (own cell + halo) ----
#pragma unroll
        for (int v = 0; v < NP; ++v) sW[v][ty + OY][tx + 2] = Wk[v];
        // switch (3D): the next plane's p and in-plane velocities of the own
        // cell and the ring cell (whose p and v_z also give its z bit)
        // (the ring cell's p and v_z there wait in sN's and the z slot of sC)
        if constexpr (SW3) {
            sN[0][ty + 1][tx + 1] = Wk1[IP];
            sN[1][ty + 1][tx + 1] = Wk1[1];
            sN[2][ty + 1][tx + 1] = Wk1[2];
            if (ringt) {
                int rr, rc;
                ring_rc(rr, rc);
                T p, vxr, vyr, vzr;
                ring_prim(kz + 1, rr, rc, p, vxr, vyr, vzr);
                sN[0][rr + 1][rc + 1] = p;
                sN[1][rr + 1][rc + 1] = vxr;
                sN[2][rr + 1][rc + 1] = vyr;
                sV[rr + 1][rc + 1] = vzr;
            }
        }
        T hcur[HPT][NP];
        if constexpr (LATE) {
            load_halo(kz, hcur);
        } else {
#pragma unroll
            for (int j = 0; j < HPT; ++j)
#pragma unroll
                for (int v = 0; v < NP; ++v) hcur[j][v] = hnext[j][v];
            if constexpr (ND == 3) load_halo(kz + 1, hnext);
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            if (hlds[j] >= 0) {
                T w[NP];
                to_prim<ND>(hcur[j], w, gm1);
                if (hflg[j] & 1) w[1] = -w[1];
                if constexpr (ND >= 2) { if (hflg[j] & 2) w[2] = -w[2]; }
#pragma unroll
                for (int v = 0; v < NP; ++v) sWf[v * RY * WX + hlds[j]] = w[v];
            }
        }
        __syncthreads();

        // ---- phase 1: x and y slopes of the tile cells and one ring beyond ----
        // Every thread takes its own cell; the ring (x: columns -1 and BX of
        // each row, y: rows -1 and BY) goes to the first threads (y) and the
        // last ones (x), so no wave carries two extra passes; the z slopes of
        // plane kz+1 (registers only) fill the wait of the other waves.
        auto slope_x = [&](int row, int col) {
#pragma unroll
            for (int v = 0; v < NP; ++v) {
                if constexpr (LIM != LIM_LEARNED)
                    sSx[v][row][col + 1] = slope_mm(sW[v][row + OY][col + 1], sW[v][row + OY][col + 2],
                                                    sW[v][row + OY][col + 3], lk);
                else
                    sSx[v][row][col + 1] = learned_slope<ND>(a, 0, v, x0 + col, y0 + row, kz);
            }
        };
        auto slope_y = [&](int row, int col) {
#pragma unroll
            for (int v = 0; v < NP; ++v) {
                if constexpr (LIM != LIM_LEARNED)
                    sSy[v][row + 1][col] = slope_mm(sW[v][row + 1][col + 2], sW[v][row + 2][col + 2],
                                                    sW[v][row + 3][col + 2], lk);
                else
                    sSy[v][row + 1][col] = learned_slope<ND>(a, 1, v, x0 + col, y0 + row, kz);
            }
        };
        // waves that also carry ring items run at raised priority so the
        // barrier that ends the phase is reached sooner
        const int wv = tid >> 6;
        // (3D only: measured 5 % faster at 256^3; the single-plane 2D blocks
        // gain nothing)
        const bool ring1 = ND == 3 && (wv < (2 * BX + 63) / 64 || wv >= (NT - 2 * BY) / 64 ||
                                       (SW && wv >= RING0 / 64 && wv < (RING0 + NRING + 63) / 64));
        const bool ring2 = ND == 3 && (wv < (BX + 63) / 64 || wv >= (NT - BY) / 64);
        if (ring1) __builtin_amdgcn_s_setprio(2);
        if constexpr (LIM != LIM_LEARNED) {
            slope_x(ty, tx);
            if constexpr (ND >= 2) slope_y(ty, tx);
        }
        if constexpr (ND == 3) {
            to_w(U2, W2, fxo, fyo, fz2);
            if constexpr (LIM != LIM_LEARNED) {
#pragma unroll
                for (int v = 0; v < NP; ++v) Sk1[v] = slope_mm(Wk[v], Wk1[v], W2[v], lk);
            } else if (own_valid && kz + 1 < nz) {
                // the z slope of plane kz+1: one plane up at the own offset
                const unsigned o = zko + colv + (unsigned)plane;
#pragma unroll
                for (int v = 0; v < NP; ++v) Sk1[v] = (T)at(a.slopes + (int64_t)(2 * NP + v) * a.vstride, o);
            } else {  // past the last plane, or a ghost column: boundary-mapped
#pragma unroll
                for (int v = 0; v < NP; ++v) Sk1[v] = learned_slope<ND>(a, 2, v, gx, gy, kz + 1);
            }
        }
        if constexpr (LIM != LIM_LEARNED) {
            if constexpr (ND >= 2) {
                if (tid < 2 * BX) slope_y(tid < BX ? -1 : BY, tid < BX ? tid : tid - BX);
            }
            if (ering >= 0) slope_x(ering >> 1, (ering & 1) ? BX : -1);
        }
        unsigned zb = 0u;  // switch: the own cell's byte (x, y bits of kz and kz + 1)
        if constexpr (SW) {
            // detector bits of plane kz: own cell and ring cell (the z bit
            // from the planes below and above; the current plane then becomes
            // the one below); the own cell's byte also keeps its x and y bits
            // of the next plane in bits 4 and 5 for its z face
            unsigned ob = bits_w(ty, tx);
            if constexpr (SW3) {
                ob |= (unsigned)shock(sC[0][ty + 1][tx + 1], Wk1[IP], sC[1][ty + 1][tx + 1], Wk1[3]) << 2;
                sC[0][ty + 1][tx + 1] = Wk[IP];
                sC[1][ty + 1][tx + 1] = Wk[3];
                ob |= bits_n() << 4;
            }
            sB[ty + 1][tx + 1] = (uint8_t)ob;
            zb = ob;
            if (ringt) {
                int rr, rc;
                ring_rc(rr, rc);
                unsigned rb = bits_w(rr, rc);
                if constexpr (SW3) {
                    rb |= (unsigned)shock(sC[0][rr + 1][rc + 1], sN[0][rr + 1][rc + 1], sC[1][rr + 1][rc + 1],
                                          sV[rr + 1][rc + 1])
                          << 2;
                    sC[0][rr + 1][rc + 1] = sW[IP][rr + OY][rc + 2];
                    sC[1][rr + 1][rc + 1] = sW[3][rr + OY][rc + 2];
                }
                sB[rr + 1][rc + 1] = (uint8_t)rb;
            }
        }
        // the z face kz+1/2 of the own column, here rather than with the x
        // and y faces: its left state's plane (W and z slope of kz) is then
        // dead before the x and y Riemann solves, which lowers their
        // register pressure
        constexpr int SV = SW ? SOLVER_HLLC : SOLVER;
        using Main = std::integral_constant<int, SV>;
        using Hll = std::integral_constant<int, SOLVER_HLL>;
        // a flagged face right after its HLLC evaluation (its inputs are
        // still in LDS or live registers, so the redo holds nothing longer)
        auto redo = [&](bool flagged, auto fn) {
            if constexpr (SW) {
                if (__builtin_amdgcn_ballot_w64(flagged) != 0ull) {
                    // the redo reads its face states again rather than keeping
                    // the first evaluation's alive through it
                    asm volatile("" ::: "memory");
                    if (flagged) fn();
                }
            }
        };
        // face z kz+1/2 of the own column (the cell of plane kz or kz + 1
        // flagged along x or y)
        auto face_z = [&](auto kind) -> bool {
            T fl[NP], fr[NP];
            face_state(Wk, Sk, hs, fl);
            face_state(Wk1, Sk1, -hs, fr);
            if constexpr (decltype(kind)::value != SV) {
                // (the redo: opaque copies, so the face states are formed
                // again instead of being kept from the first evaluation)
#pragma unroll
                for (int v = 0; v < NP; ++v) asm volatile("" : "+v"(fl[v]), "+v"(fr[v]));
            }
            riemann<ND, 2, decltype(kind)::value>(fl, fr, Fhi, sg, igm1);
            if constexpr (SW3) return ((zb | (zb >> 4)) & 3u) != 0u;
            return false;
        };
        if constexpr (ND == 3) redo(face_z(Main{}), [&] { (void)face_z(Hll{}); });
        if (ring1) __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        if (ring2) __builtin_amdgcn_s_setprio(3);

        // ---- phase 2: x and y face fluxes, each face once ----
        // own faces (the low x and y face of the own cell), then the ring:
        // face column BX (last threads) and face row BY (first threads).  The
        // switch evaluates HLLC at every face and notes the faces whose cells
        // carry a transverse shock bit; those are evaluated again with HLL
        // right after, in a branch the wavefront skips when none of its faces
        // is flagged
        // face x at (row, col) between cells col-1 and col; returns whether
        // the switch wants HLL there (either cell flagged along y or z)
        auto face_x = [&](int row, int col, auto kind) -> bool {
            T wl[NP], wr[NP], fl[NP];
#pragma unroll
            for (int v = 0; v < NP; ++v) {
                wl[v] = sW[v][row + OY][col + 1] + hs * sSx[v][row][col];
                wr[v] = sW[v][row + OY][col + 2] - hs * sSx[v][row][col + 1];
            }
            riemann<ND, 0, decltype(kind)::value>(wl, wr, fl, sg, igm1);
#pragma unroll
            for (int v = 0; v < NP; ++v) sFx[v][row][col] = fl[v];
            if constexpr (SW) return ((sB[row + 1][col] | sB[row + 1][col + 1]) & 6u) != 0u;
            return false;
        };
        // face y (either cell flagged along x or z)
        auto face_y = [&](int row, int col, auto kind) -> bool {
            T wl[NP], wr[NP], fl[NP];
#pragma unroll
            for (int v = 0; v < NP; ++v) {
                wl[v] = sW[v][row + 1][col + 2] + hs * sSy[v][row][col];
                wr[v] = sW[v][row + 2][col + 2] - hs * sSy[v][row + 1][col];
            }
            riemann<ND, 1, decltype(kind)::value>(wl, wr, fl, sg, igm1);
#pragma unroll
            for (int v = 0; v < NP; ++v) sFy[v][row][col] = fl[v];
            if constexpr (SW) return ((sB[row][col + 1] | sB[row + 1][col + 1]) & 5u) != 0u;
            return false;
        };
        const int fe = tid - (NT - BY);  // x ring face of the last threads
        // the scheduling barriers keep the solver instances from being
        // interleaved, which would only raise register pressure
        redo(face_x(ty, tx, Main{}), [&] { (void)face_x(ty, tx, Hll{}); });
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (ND >= 2) redo(face_y(ty, tx, Main{}), [&] { (void)face_y(ty, tx, Hll{}); });
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (ND >= 2) {
            if (tid < BX) redo(face_y(BY, tid, Main{}), [&] { (void)face_y(BY, tid, Hll{}); });
        }
        if (fe >= 0) redo(face_x(fe, BX, Main{}), [&] { (void)face_x(fe, BX, Hll{}); });
        if (ring2) __builtin_amdgcn_s_setprio(0);
        __syncthreads();

        // ---- phase 3: divergence, source, Runge-Kutta combination ----
        // stage 1: U + dt L; stage 2: (U^n + U^(1) + dt L) / 2, with the
        // factors dt / dq (dt / (2 dq)) of every face-flux difference uniform
        T out[NP];
        if constexpr (STAGE == 1) {
#pragma unroll
            for (int v = 0; v < NP; ++v) out[v] = Uk[v];
        } else {
            if constexpr (LATE) {
#pragma unroll
                for (int v = 0; v < NP; ++v) u0[v] = own_valid ? at(u0p[v], zko + colv) : T(0);
            }
#pragma unroll
            for (int v = 0; v < NP; ++v) out[v] = T(0.5) * (u0[v] + Uk[v]);
        }
#pragma unroll
        for (int v = 0; v < NP; ++v) out[v] += cdt[0] * (sFx[v][ty][tx] - sFx[v][ty][tx + 1]);
        if constexpr (ND >= 2) {
#pragma unroll
            for (int v = 0; v < NP; ++v) out[v] += cdt[1] * (sFy[v][ty][tx] - sFy[v][ty + 1][tx]);
        }
        if constexpr (ND == 3) {
#pragma unroll
            for (int v = 0; v < NP; ++v) out[v] += cdt[2] * (Flo[v] - Fhi[v]);
        }
        if (grav) {
            // uniform acceleration: momentum += rho a, energy += S . a
            T pw = T(0);
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                out[1 + d] += Uk[0] * cacc[d];
                pw += Uk[1 + d] * cacc[d];
            }
            out[IP] += pw;
        }
        if (own_valid) {
            const unsigned c = zko + colv;
#pragma unroll
            for (int v = 0; v < NP; ++v) *(T *)((char *)uout[v] + c * (unsigned)sizeof(T)) = out[v];
            if constexpr (STAGE == 2) {
                // CFL rate of the new state: max_q (|v_q| + c) / dq
                T wo[NP];
                bad |= !to_prim<ND>(out, wo, gm1);
                const T cs = sound_(gamma, wo[IP], wo[0]);
                if (cubic) {
                    T vm = fabs(wo[1]);
#pragma unroll
                    for (int d = 1; d < ND; ++d) vm = fmax(vm, fabs(wo[1 + d]));
                    rate = fmax(rate, (vm + cs) * a.idx[0]);
                } else {
#pragma unroll
                    for (int d = 0; d < ND; ++d) rate = fmax(rate, (fabs(wo[1 + d]) + cs) * a.idx[d]);
                }
            }
        }
    };

    if constexpr (ND == 3) {
        for (int it = 0; it < nplanes; it += 3) {
            body(it, WA, WB, WC, UA, UB, UC, SA, SB, FA, FB);
            if (it + 1 < nplanes) body(it + 1, WB, WC, WA, UB, UC, UA, SB, SC, FB, FC);
            if (it + 2 < nplanes) body(it + 2, WC, WA, WB, UC, UA, UB, SC, SA, FC, FA);
        }
    } else {
        body(0, WA, WB, WC, UA, UB, UC, SA, SB, FA, FB);
    }

    if (bad) atomicOr(&a.ctl->err, 1u);
    if constexpr (STAGE == 2) {
        // wave max, block max in LDS, one atomic per block into slot
        // blockIdx % RATE_SLOTS (positive doubles order as uint64)
        __shared__ double sRate[NT / 64];
        double r = (double)rate;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off, 64));
        if ((tid & 63) == 0) sRate[tid >> 6] = r;
        __syncthreads();
        if (tid == 0) {
            double m = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) m = fmax(m, sRate[w]);
            if (m > 0.0)
                atomicMax(&a.ctl->rate[a.parity ^ 1][blockIdx.x % RATE_SLOTS], (unsigned long long)__double_as_longlong(m));
        }
    }
}

template <int ND, typename T, int SOLVER, int STAGE, int LIM, int BX, int BY>
hipError_t launch_one(const LaunchCfg &cfg, StageArgs<T> a, hipStream_t s)
{
    a.tiles_x = (int)((a.n[0] + BX - 1) / BX);
    a.tiles_y = ND >= 2 ? (int)((a.n[1] + BY - 1) / BY) : 1;
    const int chunks = ND == 3 ? (int)((a.n[2] + cfg.zchunk - 1) / cfg.zchunk) : 1;
    a.ntiles = a.tiles_x * a.tiles_y * chunks;
    int64_t blocks = a.ntiles;
    a.nbfwg = 0;
    if constexpr (LIM == LIM_THETA_PADDED) {
        if (a.bf.nbox > 0) {
            if (a.bf.nbox > 2 || a.dt_mode != DT_PTR || !a.dt_dev) return hipErrorInvalidValue;
            int most = 0;
            for (int k = 0; k < a.bf.nbox; ++k)
                for (int q = 0; q < ND; ++q) {
                    const int r1 = q == 0 ? 1 : 0, r2 = q == 2 ? 1 : 2;
                    most = most > a.bf.b[k].n[r1] * a.bf.b[k].n[r2] ? most : a.bf.b[k].n[r1] * a.bf.b[k].n[r2];
                }
            a.bf.blocks = (most + BX * BY - 1) / (BX * BY);
            a.nbfwg = a.bf.nbox * ND * 2 * a.bf.blocks;
            blocks += a.nbfwg;
        }
        const int rb = (a.ride.cells + BX * BY - 1) / (BX * BY);
        a.ride.blocks = (a.ride.cells > 0 || a.ride.ck.c) ? (rb > 1 ? rb : 1) : 0;
        blocks += a.ride.blocks;
    }
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_stage<ND, T, SOLVER, STAGE, LIM, BX, BY>), dim3((unsigned)blocks), dim3(BX, BY, 1), 0, s, a);
    return hipGetLastError();
}

// Supported plane tiles (BX x BY threads): 64x8, 32x16 (FP32), 64x4, 32x8.
template <int ND, typename T, int SOLVER, int STAGE, int LIM>
hipError_t launch_by(const LaunchCfg &cfg, const StageArgs<T> &a, hipStream_t s)
{
    if constexpr (ND == 1) {
        return launch_one<ND, T, SOLVER, STAGE, LIM, 64, 1>(cfg, a, s);
    } else {
        if constexpr (sizeof(T) == 4) {
            if (cfg.bx == 32 && cfg.by == 16) return launch_one<ND, T, SOLVER, STAGE, LIM, 32, 16>(cfg, a, s);
        }
        if (cfg.bx == 32 && cfg.by == 8) return launch_one<ND, T, SOLVER, STAGE, LIM, 32, 8>(cfg, a, s);
        if (cfg.bx == 64 && cfg.by == 4) return launch_one<ND, T, SOLVER, STAGE, LIM, 64, 4>(cfg, a, s);
        return launch_one<ND, T, SOLVER, STAGE, LIM, 64, 8>(cfg, a, s);
    }
}

template <int ND, typename T, int SOLVER, int STAGE>
hipError_t launch_lim(int limiter, const LaunchCfg &cfg, const StageArgs<T> &a, hipStream_t s)
{
    if constexpr (sizeof(T) == 4) {
        if (limiter == LIM_LEARNED) return launch_by<ND, T, SOLVER, STAGE, LIM_LEARNED>(cfg, a, s);
    }
    if constexpr (SOLVER != SOLVER_HLLC_SWITCH) {
        if (limiter == LIM_THETA_PADDED) return launch_by<ND, T, SOLVER, STAGE, LIM_THETA_PADDED>(cfg, a, s);
    } else {
        if (limiter == LIM_THETA_PADDED) return hipErrorInvalidValue;
    }
    return launch_by<ND, T, SOLVER, STAGE, LIM_THETA>(cfg, a, s);
}

template <int ND, typename T>
hipError_t launch_nd(int solver, int stage, int limiter, const LaunchCfg &cfg, const StageArgs<T> &a,
                     hipStream_t s)
{
    if (solver == SOLVER_HLL) {
        return stage == 1 ? launch_lim<ND, T, 0, 1>(limiter, cfg, a, s) : launch_lim<ND, T, 0, 2>(limiter, cfg, a, s);
    }
    if constexpr (ND >= 2) {  // in 1D no face is transverse to anything: the switch is HLLC
        if (solver == SOLVER_HLLC_SWITCH)
            return stage == 1 ? launch_lim<ND, T, 2, 1>(limiter, cfg, a, s) : launch_lim<ND, T, 2, 2>(limiter, cfg, a, s);
    }
    return stage == 1 ? launch_lim<ND, T, 1, 1>(limiter, cfg, a, s) : launch_lim<ND, T, 1, 2>(limiter, cfg, a, s);
}

}  // namespace

template <typename T>
hipError_t launch_stage(int ndim, int solver, int stage, int limiter, const LaunchCfg &cfg,
                        const StageArgs<T> &a, hipStream_t s)
{
    switch (ndim) {
    case 1: return launch_nd<1, T>(solver, stage, limiter, cfg, a, s);
    case 2: return launch_nd<2, T>(solver, stage, limiter, cfg, a, s);
    default: return launch_nd<3, T>(solver, stage, limiter, cfg, a, s);
    }
}

template hipError_t launch_stage<float>(int, int, int, int, const LaunchCfg &, const StageArgs<float> &, hipStream_t);
template hipError_t launch_stage<double>(int, int, int, int, const LaunchCfg &, const StageArgs<double> &, hipStream_t);

}  // namespace hy
