// shock.hip -- the shock detector behind the HLLC -> HLL switch.
//
// HLLC resolves contacts and shear layers sharply, but a shock running along
// a grid axis can decouple neighbouring rows of cells (odd-even decoupling);
// the method therefore uses the more diffusive HLL flux in the immediate
// vicinity of a shock, at the faces transverse to its direction of motion
// (Sec. 3.2, which gives no detector).  Detector used here: a cell is in a
// shock moving along q when the pressures of its two neighbours along q
// differ by more than eps = 0.5 of the smaller one and the velocity along q
// decreases across the cell (compression).  The stage kernel then takes HLL
// at a face normal to r when either of its cells carries a bit q != r.
//
// Two passes.  The first evaluates the detector (the
// neighbours' primitives recovered from the conserved state; ghosts by the
// boundary map: periodic wrap, outflow copy, reflecting mirror with the
// normal velocity negated).  The second turns the detector bits into face
// decisions, so the stage kernel reads one byte per face: bit q (q < 3) of a
// cell is the decision for its low face along q (between cell - e_q, a ghost
// at a wall, and the cell); bit 3 + q is the decision for the high face of a
// cell at the high end of a non-periodic dimension q (its other cell is the
// ghost, whose transverse bits are those of the cell it mirrors or copies).
#include "hy_internal.h"

namespace hy {
namespace {

struct Bc3 {
    int v[3][2];
};

// Source cell of index i along a dimension of n cells; flip is set when the
// source is a mirror image.  Indices far outside the ghost range (only met by
// the unused threads of partial tiles) are clamped into the array.
__device__ __forceinline__ int map_nb(int i, int n, int lo, int hi, bool &flip)
{
    if (i >= 0 && i < n) return i;
    int m;
    if (i < 0) {
        if (lo == BC_PERIODIC) m = i + n;
        else if (lo == BC_OUTFLOW) m = 0;
        else { m = -1 - i; flip = true; }
    } else {
        if (hi == BC_PERIODIC) m = i - n;
        else if (hi == BC_OUTFLOW) m = n - 1;
        else { m = 2 * n - 1 - i; flip = true; }
    }
    return m < 0 ? 0 : (m >= n ? n - 1 : m);
}

// Detector pass: a workgroup owns a 64 x 4 column tile of the x-y plane and
// marches along z over a chunk of planes.  Per plane, the pressure and the
// in-plane velocities of the tile and a one-cell ring go to LDS (each cell
// converted once); the own column's pressure and v_z of the planes below and
// above live in registers.  Offsets are 32-bit (the library keeps a
// variable's array below 4 GiB).
constexpr int DT_X = 64, DT_Y = 4, DT_Z = 16;

template <int ND, typename T>
__global__ void __launch_bounds__(DT_X * DT_Y) k_shock_flags(const T *__restrict__ u, uint8_t *__restrict__ flags,
                                                             int nx, int ny, int nz, int64_t vstride, Bc3 bc, T gm1,
                                                             T eps, int tiles_x, int tiles_y)
{
    constexpr int WX = DT_X + 2, WY = DT_Y + 2, NV = ND + 2;
    __shared__ T sP[WY][WX], sVx[DT_Y][WX], sVy[WY][DT_X];
    const int tx = threadIdx.x % DT_X, ty = threadIdx.x / DT_X, tid = threadIdx.x;
    const int bxi = blockIdx.x % tiles_x, rest = blockIdx.x / tiles_x;
    const int byi = rest % tiles_y, bzi = rest / tiles_y;
    const int x0 = bxi * DT_X, y0 = byi * DT_Y, z0 = bzi * DT_Z;
    const int z1 = min(z0 + DT_Z, nz);
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const T *uv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) uv[v] = u + (int64_t)v * vstride;

    // pressure and one velocity component of the cell at offset o (flip:
    // the component is the normal velocity of a mirror image); in FP32 the
    // reciprocal of D is the 1-ulp hardware one, as in the stage kernel (the
    // detector only compares, and its decisions are tested away from the
    // threshold)
    auto prim = [&](unsigned o, int comp, bool flip, T &pp, T &vv) {
        const T D = uv[0][o];
        T ir;
        if constexpr (sizeof(T) == 4) ir = __builtin_amdgcn_rcpf(D);
        else ir = T(1) / D;
        T s2 = T(0), sc = T(0);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const T S = uv[1 + d][o];
            s2 += S * S;
            if (d == comp) sc = S;
        }
        pp = gm1 * (uv[NV - 1][o] - T(0.5) * s2 * ir);
        vv = (flip ? -sc : sc) * ir;
    };
    auto map = [&](int i, int n, int q, bool &flip) -> int {
        return map_nb(i, n, bc.v[q][0], bc.v[q][1], flip);
    };

    // own column; in a partial tile the first position past the end is the
    // ghost cell the last real cell needs, further ones are never used
    bool fx = false, fy = false;
    const int mx = map(x0 + tx, nx, 0, fx);
    const int my = map(y0 + ty, ny, 1, fy);
    const unsigned col = (unsigned)my * (unsigned)nx + (unsigned)mx;
    const bool own = x0 + tx < nx && y0 + ty < ny;

    // all primitives the detector needs of the own column at plane z (fz:
    // the plane is a mirror image along z): p, v_x, v_y, v_z
    auto column = [&](int z, T (&c)[4]) {
        bool fz = false;
        const int mz = ND == 3 ? map(z, nz, 2, fz) : 0;
        const unsigned o = (unsigned)mz * plane + col;
        const T D = uv[0][o];
        T ir;
        if constexpr (sizeof(T) == 4) ir = __builtin_amdgcn_rcpf(D);
        else ir = T(1) / D;
        T s2 = T(0), S[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            S[d] = uv[1 + d][o];
            s2 += S[d] * S[d];
        }
        c[0] = gm1 * (uv[NV - 1][o] - T(0.5) * s2 * ir);
        c[1] = (fx ? -S[0] : S[0]) * ir;
        c[2] = (fy ? -S[1] : S[1]) * ir;
        c[3] = (fz ? -S[2] : S[2]) * ir;
    };
    // ring item of this thread at plane z: the x halo columns -1 and DT_X of
    // every row, then the y halo rows -1 and DT_Y (pressure and the velocity
    // normal to the halo side)
    const int nring = 2 * DT_Y + 2 * DT_X;
    auto ring = [&](int z, T &pp, T &vv) {
        const unsigned zo = (unsigned)z * plane;
        bool f = false, g = false;
        if (tid < 2 * DT_Y) {
            const int r = tid >> 1, side = tid & 1;
            const int hx = map(x0 + (side ? DT_X : -1), nx, 0, f);
            const int hy = map(y0 + r, ny, 1, g);
            prim(zo + (unsigned)hy * (unsigned)nx + (unsigned)hx, 0, f, pp, vv);
        } else {
            const int e = tid - 2 * DT_Y, c = e >> 1, side = e & 1;
            const int hy = map(y0 + (side ? DT_Y : -1), ny, 1, f);
            const int hx = map(x0 + c, nx, 0, g);
            prim(zo + (unsigned)hy * (unsigned)nx + (unsigned)hx, 1, f, pp, vv);
        }
    };

    // plane z0 and the z window below it; every later plane is loaded one
    // iteration ahead, so its latency overlaps the current plane's work
    T cm[4] = {T(0), T(0), T(0), T(0)}, c0[4];
    if constexpr (ND == 3) column(z0 - 1, cm);
    column(z0, c0);
    T hp = T(0), hv = T(0);
    const bool has_ring = tid < nring && (ND >= 2 || tid < 2 * DT_Y);
    if (has_ring) ring(z0, hp, hv);
    for (int z = z0; z < z1; ++z) {
        sP[ty + 1][tx + 1] = c0[0];
        sVx[ty][tx + 1] = c0[1];
        sVy[ty + 1][tx] = c0[2];
        if (has_ring) {
            if (tid < 2 * DT_Y) {
                const int r = tid >> 1, side = tid & 1;
                sP[r + 1][side ? DT_X + 1 : 0] = hp;
                sVx[r][side ? DT_X + 1 : 0] = hv;
            } else {
                const int e = tid - 2 * DT_Y, c = e >> 1, side = e & 1;
                sP[side ? DT_Y + 1 : 0][c + 1] = hp;
                sVy[side ? DT_Y + 1 : 0][c] = hv;
            }
        }
        T cp[4] = {T(0), T(0), T(0), T(0)};
        if constexpr (ND == 3) {
            column(z + 1, cp);
            if (has_ring && z + 1 < z1) ring(z + 1, hp, hv);
        }
        __syncthreads();
        unsigned bits = 0;
        {
            const T pa = sP[ty + 1][tx], pb = sP[ty + 1][tx + 2];
            if (fabs(pb - pa) > eps * fmin(pa, pb) && sVx[ty][tx + 2] - sVx[ty][tx] < T(0)) bits |= 1u;
        }
        if constexpr (ND >= 2) {
            const T pa = sP[ty][tx + 1], pb = sP[ty + 2][tx + 1];
            if (fabs(pb - pa) > eps * fmin(pa, pb) && sVy[ty + 2][tx] - sVy[ty][tx] < T(0)) bits |= 2u;
        }
        if constexpr (ND == 3) {
            if (fabs(cp[0] - cm[0]) > eps * fmin(cm[0], cp[0]) && cp[3] - cm[3] < T(0)) bits |= 4u;
        }
        if (own) flags[(unsigned)z * plane + col] = (uint8_t)bits;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            cm[k] = c0[k];
            c0[k] = cp[k];
        }
        __syncthreads();
    }
}

// Face decisions: one thread per cell (grid: x blocks by y by z).  The low
// neighbour along q is the cell itself shifted by one, a ghost only at a low
// wall.
template <int ND>
__global__ void __launch_bounds__(256) k_face_decisions(const uint8_t *__restrict__ det, uint8_t *__restrict__ faces,
                                                        int nx, int ny, int nz, Bc3 bc)
{
    const int x = (int)(blockIdx.x * 256 + threadIdx.x);
    if (x >= nx) return;
    const int pos[3] = {x, (int)blockIdx.y, (int)blockIdx.z};
    const int ext[3] = {nx, ny, nz};
    const unsigned stride[3] = {1u, (unsigned)nx, (unsigned)nx * (unsigned)ny};
    const unsigned c = ((unsigned)pos[2] * (unsigned)ny + (unsigned)pos[1]) * (unsigned)nx + (unsigned)x;
    const unsigned own = det[c];
    unsigned out = 0;
#pragma unroll
    for (int q = 0; q < ND; ++q) {
        const unsigned mask = ~(1u << q) & 7u;
        unsigned lo;
        if (pos[q] > 0) {
            lo = det[c - stride[q]];
        } else {
            bool flip = false;
            const int m = map_nb(-1, ext[q], bc.v[q][0], bc.v[q][1], flip);
            lo = det[c + (unsigned)m * stride[q]];
        }
        if ((own | lo) & mask) out |= 1u << q;
        if (pos[q] == ext[q] - 1 && bc.v[q][1] != BC_PERIODIC && (own & mask)) out |= 8u << q;
    }
    faces[c] = (uint8_t)out;
}

}  // namespace

template <typename T>
hipError_t launch_shock_flags(const T *u, uint8_t *det, uint8_t *flags, const int64_t n[3], int64_t vstride, int ndim,
                              const int bc[3][2], T gm1, T eps, hipStream_t s)
{
    Bc3 b;
    for (int q = 0; q < 3; ++q) {
        b.v[q][0] = bc[q][0];
        b.v[q][1] = bc[q][1];
    }
    const int nx = (int)n[0], ny = (int)n[1], nz = (int)n[2];
    const dim3 grid((unsigned)((n[0] + 255) / 256), (unsigned)n[1], (unsigned)n[2]);
    const int tx = (nx + DT_X - 1) / DT_X, ty = (ny + DT_Y - 1) / DT_Y, tz = (nz + DT_Z - 1) / DT_Z;
    const dim3 tgrid((unsigned)((int64_t)tx * ty * tz));
    switch (ndim) {
    case 2:
        hipLaunchKernelGGL((k_shock_flags<2, T>), tgrid, dim3(DT_X * DT_Y), 0, s, u, det, nx, ny, nz, vstride, b, gm1,
                           eps, tx, ty);
        hipLaunchKernelGGL((k_face_decisions<2>), grid, dim3(256), 0, s, det, flags, nx, ny, nz, b);
        break;
    case 3:
        hipLaunchKernelGGL((k_shock_flags<3, T>), tgrid, dim3(DT_X * DT_Y), 0, s, u, det, nx, ny, nz, vstride, b, gm1,
                           eps, tx, ty);
        hipLaunchKernelGGL((k_face_decisions<3>), grid, dim3(256), 0, s, det, flags, nx, ny, nz, b);
        break;
    default:  // 1D: no transverse faces, nothing to decide
        break;
    }
    return hipGetLastError();
}

template hipError_t launch_shock_flags<float>(const float *, uint8_t *, uint8_t *, const int64_t[3], int64_t, int,
                                              const int[3][2], float, float, hipStream_t);
template hipError_t launch_shock_flags<double>(const double *, uint8_t *, uint8_t *, const int64_t[3], int64_t, int,
                                               const int[3][2], double, double, hipStream_t);

}  // namespace hy
