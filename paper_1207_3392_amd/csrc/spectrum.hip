// spectrum.hip -- the kinetic-energy spectrum of the Kelvin-Helmholtz
// analysis (Sec. 4.3.1) on the device, for a 2D patch of N x N cells (N a
// power of two up to 8192) on a square box of side L.
//
// Both velocity components go through one complex transform: with
// z = sqrt(rho) (v_x + i v_y) = (S_x + i S_y) / sqrt(D) and Z its discrete
// Fourier transform, the transforms A, B of the real fields sqrt(rho) v_x,
// sqrt(rho) v_y satisfy |A(k)|^2 + |B(k)|^2 = (|Z(k)|^2 + |Z(-k)|^2) / 2, and
// a shell of |k| holds k and -k together, so a shell's sum of |A|^2 + |B|^2
// is its sum of |Z|^2.  The transform is FP64: radix-2
// decimation-in-frequency FFTs of whole rows staged in LDS (output in
// bit-reversed order, which the binning undoes by index), with a tiled
// transpose between the x and the y pass.  The squared magnitudes are
// binned on the integer shell nearest to |n| (n the integer wavevector) as
// 64-bit fixed-point sums at a power-of-two scale taken from the total
// (Parseval), so the shell sums are exact integer additions whose result
// does not depend on the order in which workgroups add.  e(s) =
// L^2 / (2 N^4 dk) * sum over the shell of |Z|^2, dk = 2 pi / L: the
// integral of rho |v|^2 / 2 over the box is sum_s e(s) dk.
#include "hy_internal.h"
#include "hy_diag.h"

#include <math.h>

namespace hy {
namespace {

constexpr int FT = 256;                  // threads of the FFT and binning workgroups
constexpr int SPEC_MAX_LOG2 = 13;        // N <= 8192: a row of FP64 complex values fits in LDS
constexpr int SPEC_ROWS_PER_BLOCK = 4;   // rows of the transformed array per binning workgroup

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// tw[t] = exp(-2 pi i t / N), t < N / 2
__global__ void __launch_bounds__(FT) k_twiddle(double2 *tw, int n)
{
    const int t = blockIdx.x * FT + threadIdx.x;
    if (t < n / 2) {
        double s, c;
        sincospi(-2.0 * (double)t / (double)n, &s, &c);
        tw[t] = make_double2(c, s);
    }
}

// One workgroup per row: stage the row in LDS (MODE 0: z from the conserved
// state, and the row's sum of |z|^2; MODE 1: a complex row), transform it
// in place, write it out in bit-reversed frequency order.
template <int L, int MODE, typename T>
__global__ void __launch_bounds__(FT) k_fft_rows(const T *u, int64_t vs, const double2 *src, double2 *dst,
                                                  const double2 *tw, double *rowsum, DevCtl *ctl)
{
    constexpr int N = 1 << L;
    __shared__ double2 x[N];
    __shared__ double red[FT];
    const int tid = threadIdx.x;
    const int64_t row = blockIdx.x;
    if constexpr (MODE == 0) {
        double acc = 0.0;
        bool bad = false;
        for (int i = tid; i < N; i += FT) {
            const int64_t c = row * N + i;
            const double D = (double)u[c], sx = (double)u[vs + c], sy = (double)u[2 * vs + c];
            bad |= !(D > 0.0);
            const double r = 1.0 / sqrt(D);
            const double2 z = make_double2(sx * r, sy * r);
            x[i] = z;
            acc += z.x * z.x + z.y * z.y;
        }
        if (bad) atomicOr(&ctl->err, 1u);
        red[tid] = acc;
        __syncthreads();
        for (int off = FT / 2; off > 0; off >>= 1) {
            if (tid < off) red[tid] += red[tid + off];
            __syncthreads();
        }
        if (tid == 0) rowsum[row] = red[0];
    } else {
        for (int i = tid; i < N; i += FT) x[i] = src[row * N + i];
        __syncthreads();
    }
    // stage s: butterflies of span 2^s inside blocks of 2^(s+1); the twiddle
    // of butterfly j of a block is exp(-2 pi i j / 2^(s+1)) = tw[j N / 2^(s+1)]
    for (int s = L - 1; s >= 0; --s) {
        const int half = 1 << s;
        for (int b = tid; b < N / 2; b += FT) {
            const int j = b & (half - 1);
            const int i0 = ((b >> s) << (s + 1)) | j;
            const int i1 = i0 + half;
            const double2 a = x[i0], c = x[i1];
            x[i0] = make_double2(a.x + c.x, a.y + c.y);
            x[i1] = cmul(make_double2(a.x - c.x, a.y - c.y), tw[j << (L - 1 - s)]);
        }
        __syncthreads();
    }
    for (int i = tid; i < N; i += FT) dst[row * N + i] = x[i];
}

// dst[c][r] = src[r][c] for an n x n array, 32 x 32 tiles through LDS
__global__ void __launch_bounds__(FT) k_transpose(const double2 *src, double2 *dst, int n)
{
    __shared__ double2 t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;
    for (int k = 0; k < 32; k += 8) {
        const int r = by + ty + k, c = bx + tx;
        if (r < n && c < n) t[ty + k][tx] = src[(int64_t)r * n + c];
    }
    __syncthreads();
    for (int k = 0; k < 32; k += 8) {
        const int r = bx + ty + k, c = by + tx;
        if (r < n && c < n) dst[(int64_t)r * n + c] = t[tx][ty + k];
    }
}

// The fixed-point scale 2^(61 - e), 2^e > sum |Z|^2 = N^2 sum |z|^2, so that
// every shell sum stays below 2^62; clears the shell sums.
__global__ void __launch_bounds__(FT) k_spec_scale(const double *rowsum, int n, double *scale,
                                                    unsigned long long *q, int nshell)
{
    __shared__ double red[FT];
    const int tid = threadIdx.x;
    double acc = 0.0;
    for (int i = tid; i < n; i += FT) acc += rowsum[i];
    red[tid] = acc;
    __syncthreads();
    for (int off = FT / 2; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        const double total = red[0] * (double)n * (double)n;
        scale[0] = (total > 0.0 && total < 1e300) ? ldexp(1.0, 61 - (ilogb(total) + 1)) : 0.0;
    }
    for (int i = tid; i < nshell; i += FT) q[i] = 0ull;
}

__device__ __forceinline__ int signed_freq(int i, int n) { return i < n / 2 ? i : i - n; }

// Element (r, c) of the twice-transformed array holds the frequency
// (bitrev(r), bitrev(c)) along (x, y): its |Z|^2 goes to the shell nearest
// to the wavevector's length, first into the workgroup's LDS sums.
__global__ void __launch_bounds__(FT) k_spec_bin(const double2 *C, int L, const double *scale,
                                                  unsigned long long *q, int nshell)
{
    __shared__ unsigned long long part[SPEC_MAX_SHELLS];
    const int tid = threadIdx.x;
    const int n = 1 << L;
    for (int i = tid; i < nshell; i += FT) part[i] = 0ull;
    __syncthreads();
    const double s = scale[0];
    const int r0 = blockIdx.x * SPEC_ROWS_PER_BLOCK;
    const int r1 = r0 + SPEC_ROWS_PER_BLOCK < n ? r0 + SPEC_ROWS_PER_BLOCK : n;
    for (int r = r0; r < r1; ++r) {
        const int fx = signed_freq((int)(__brev((unsigned)r) >> (32 - L)), n);
        for (int c = tid; c < n; c += FT) {
            const int fy = signed_freq((int)(__brev((unsigned)c) >> (32 - L)), n);
            const double2 z = C[(int64_t)r * n + c];
            const unsigned long long v = (unsigned long long)((z.x * z.x + z.y * z.y) * s);
            const int sh = (int)floor(sqrt((double)(fx * fx + fy * fy)) + 0.5);
            if (v) atomicAdd(&part[sh], v);
        }
    }
    __syncthreads();
    for (int i = tid; i < nshell; i += FT)
        if (part[i]) atomicAdd(&q[i], part[i]);
}

__global__ void __launch_bounds__(FT) k_spec_final(const unsigned long long *q, const double *scale, int nshell,
                                                    int n, double box, double *e)
{
    const int i = blockIdx.x * FT + threadIdx.x;
    if (i >= nshell) return;
    const double s = scale[0];
    const double n2 = (double)n * (double)n;
    const double dk = 2.0 * M_PI / box;
    e[i] = s > 0.0 ? (double)q[i] / s * (0.5 * box * box / (n2 * n2) / dk) : 0.0;
}

template <int L, int MODE, typename T>
void fft_rows_launch(const T *u, int64_t vs, const double2 *src, double2 *dst, const double2 *tw, double *rowsum,
                     DevCtl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL((k_fft_rows<L, MODE, T>), dim3(1u << L), dim3(FT), 0, s, u, vs, src, dst, tw, rowsum, ctl);
}

template <int MODE, typename T>
hipError_t fft_rows(int L, const T *u, int64_t vs, const double2 *src, double2 *dst, const double2 *tw,
                    double *rowsum, DevCtl *ctl, hipStream_t s)
{
    switch (L) {
#define HY_FFT_CASE(l) \
    case l: fft_rows_launch<l, MODE, T>(u, vs, src, dst, tw, rowsum, ctl, s); break;
        HY_FFT_CASE(1) HY_FFT_CASE(2) HY_FFT_CASE(3) HY_FFT_CASE(4) HY_FFT_CASE(5) HY_FFT_CASE(6)
        HY_FFT_CASE(7) HY_FFT_CASE(8) HY_FFT_CASE(9) HY_FFT_CASE(10) HY_FFT_CASE(11) HY_FFT_CASE(12)
        HY_FFT_CASE(13)
#undef HY_FFT_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

int spectrum_shells(int n) { return (int)floor(sqrt(2.0) * (double)(n / 2) + 0.5) + 1; }

size_t spectrum_workspace_bytes(int n)
{
    const size_t nn = (size_t)n * (size_t)n;
    const size_t sh = (size_t)spectrum_shells(n);
    return 256 + 2 * align256(nn * sizeof(double2)) + align256((size_t)(n / 2) * sizeof(double2)) +
           align256((size_t)n * sizeof(double)) + align256(sizeof(double)) + align256(sh * 8) + align256(sh * 8);
}

template <typename T>
hipError_t launch_spectrum(const T *u, int64_t vstride, int n, double box, void *ws, double **e_dev, DevCtl *ctl,
                           hipStream_t s)
{
    int L = 0;
    while ((1 << L) < n) ++L;
    if (n < 2 || (1 << L) != n || L > SPEC_MAX_LOG2) return hipErrorInvalidValue;
    const size_t nn = (size_t)n * (size_t)n;
    const int nshell = spectrum_shells(n);
    char *p = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    double2 *A = (double2 *)p;
    p += align256(nn * sizeof(double2));
    double2 *B = (double2 *)p;
    p += align256(nn * sizeof(double2));
    double2 *tw = (double2 *)p;
    p += align256((size_t)(n / 2) * sizeof(double2));
    double *rowsum = (double *)p;
    p += align256((size_t)n * sizeof(double));
    double *scale = (double *)p;
    p += align256(sizeof(double));
    unsigned long long *q = (unsigned long long *)p;
    p += align256((size_t)nshell * 8);
    double *e = (double *)p;
    *e_dev = e;

    hipLaunchKernelGGL(k_twiddle, dim3((unsigned)((n / 2 + FT - 1) / FT)), dim3(FT), 0, s, tw, n);
    hipError_t err = fft_rows<0, T>(L, u, vstride, nullptr, A, tw, rowsum, ctl, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_spec_scale, dim3(1), dim3(FT), 0, s, rowsum, n, scale, q, nshell);
    const unsigned tiles = (unsigned)((n + 31) / 32);
    hipLaunchKernelGGL(k_transpose, dim3(tiles, tiles), dim3(32, 8), 0, s, A, B, n);
    err = fft_rows<1, T>(L, nullptr, 0, B, A, tw, nullptr, ctl, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_spec_bin, dim3((unsigned)((n + SPEC_ROWS_PER_BLOCK - 1) / SPEC_ROWS_PER_BLOCK)), dim3(FT),
                       0, s, A, L, scale, q, nshell);
    hipLaunchKernelGGL(k_spec_final, dim3((unsigned)((nshell + FT - 1) / FT)), dim3(FT), 0, s, q, scale, nshell, n,
                       box, e);
    return hipGetLastError();
}

template hipError_t launch_spectrum<float>(const float *, int64_t, int, double, void *, double **, DevCtl *,
                                           hipStream_t);
template hipError_t launch_spectrum<double>(const double *, int64_t, int, double, void *, double **, DevCtl *,
                                            hipStream_t);

}  // namespace hy
