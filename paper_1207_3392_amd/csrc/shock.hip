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
// One thread per cell; the neighbours' primitives are recovered from the
// conserved state (ghosts by the boundary map: periodic wrap, outflow copy,
// reflecting mirror with the normal velocity negated).  The pass reads the
// state once through the caches and writes one byte per cell.
#include "hy_internal.h"

namespace hy {
namespace {

struct Bc3 {
    int v[3][2];
};

__device__ __forceinline__ int64_t map_nb(int64_t i, int64_t n, int lo, int hi, bool &flip)
{
    if (i >= 0 && i < n) return i;
    if (i < 0) {
        if (lo == BC_PERIODIC) return i + n;
        if (lo == BC_OUTFLOW) return 0;
        flip = true;
        return -1 - i;
    }
    if (hi == BC_PERIODIC) return i - n;
    if (hi == BC_OUTFLOW) return n - 1;
    flip = true;
    return 2 * n - 1 - i;
}

template <int ND, typename T>
__global__ void __launch_bounds__(256) k_shock_flags(const T *__restrict__ u, uint8_t *__restrict__ flags, int64_t nx,
                                                     int64_t ny, int64_t nz, int64_t vstride, Bc3 bc, T gm1, T eps)
{
    const int64_t ncell = nx * ny * nz;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= ncell) return;
    const int64_t pos[3] = {c % nx, (c / nx) % ny, c / (nx * ny)};
    const int64_t ext[3] = {nx, ny, nz};
    const int64_t stride[3] = {1, nx, nx * ny};
    unsigned bits = 0;
#pragma unroll
    for (int q = 0; q < ND; ++q) {
        T p[2], vq[2];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            bool flip = false;
            const int64_t m = map_nb(pos[q] + (side ? 1 : -1), ext[q], bc.v[q][0], bc.v[q][1], flip);
            const int64_t cc = c + (m - pos[q]) * stride[q];
            const T D = u[cc];
            T s2 = T(0), sq = T(0);
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                const T S = u[cc + (1 + d) * vstride];
                s2 += S * S;
                if (d == q) sq = S;
            }
            const T G = u[cc + (ND + 1) * vstride];
            p[side] = gm1 * (G - T(0.5) * s2 / D);
            vq[side] = (flip ? -sq : sq) / D;
        }
        if (fabs(p[1] - p[0]) > eps * fmin(p[0], p[1]) && vq[1] - vq[0] < T(0)) bits |= 1u << q;
    }
    flags[c] = (uint8_t)bits;
}

}  // namespace

template <typename T>
hipError_t launch_shock_flags(const T *u, uint8_t *flags, const int64_t n[3], int64_t vstride, int ndim,
                              const int bc[3][2], T gm1, T eps, hipStream_t s)
{
    Bc3 b;
    for (int q = 0; q < 3; ++q) {
        b.v[q][0] = bc[q][0];
        b.v[q][1] = bc[q][1];
    }
    const int64_t ncell = n[0] * n[1] * n[2];
    const dim3 grid((unsigned)((ncell + 255) / 256));
    switch (ndim) {
    case 1: hipLaunchKernelGGL((k_shock_flags<1, T>), grid, dim3(256), 0, s, u, flags, n[0], n[1], n[2], vstride, b, gm1, eps); break;
    case 2: hipLaunchKernelGGL((k_shock_flags<2, T>), grid, dim3(256), 0, s, u, flags, n[0], n[1], n[2], vstride, b, gm1, eps); break;
    default: hipLaunchKernelGGL((k_shock_flags<3, T>), grid, dim3(256), 0, s, u, flags, n[0], n[1], n[2], vstride, b, gm1, eps); break;
    }
    return hipGetLastError();
}

template hipError_t launch_shock_flags<float>(const float *, uint8_t *, const int64_t[3], int64_t, int,
                                              const int[3][2], float, float, hipStream_t);
template hipError_t launch_shock_flags<double>(const double *, uint8_t *, const int64_t[3], int64_t, int,
                                               const int[3][2], double, double, hipStream_t);

}  // namespace hy
