// mlp.hip -- the learned slope limiter on gfx950 matrix cores.
//
// The network (4 -> 32 -> 32 -> 1, ReLU) replaces the generalised minmod of
// eq. MinMod.  Its inputs are the four one-sided differences of a 5-cell
// stencil of one primitive variable along one dimension, divided by
// s = max|d| + 1e-12 (|w_c| + 1e-30); its output times s is clamped to the TVD
// region 0 <= sign(D) sigma <= 2 min(|D-|, |D+|) (zero where the central
// differences D-, D+ disagree in sign), so the result never leaves the region
// that contains minmod and the monotonized-central limiter.
//
// Matrix layers run as bf16 MFMA (v_mfma_f32_16x16x16_bf16) with FP32
// accumulation; biases enter as the accumulator input; layer 3 (32 -> 1) is an
// FP32 dot product.  One wave evaluates 64 stencils at a time, one per lane,
// in the transposed orientation H^T = W X^T so that each layer's output
// registers are already the next layer's operand layout:
//   lane l = (grp = l / 16, col = l % 16) owns stencil (batch grp, column col);
//   layer 1: for each batch g, A = W1 placed in K-group g (zeros elsewhere),
//            B = the lanes' own bf16 inputs (K-group = grp), C = b1;
//   layer 2: A = W2 blocks, B = relu(H1) as bf16, C = b2;
//   layer 3: per-lane partial dot products, summed over the four lane groups.
#include "hy_internal.h"
#include "hy_mlp.h"

#include <hip/hip_bf16.h>
#include <cstring>

namespace hy {

void mlp_pack(const float *flat, MlpDevice *out)
{
    std::memset(out, 0, sizeof(*out));
    const float *p = flat;
    std::memcpy(out->w1, p, sizeof(out->w1)); p += MLP_H * MLP_IN;
    std::memcpy(out->b1, p, sizeof(out->b1)); p += MLP_H;
    std::memcpy(out->w2, p, sizeof(out->w2)); p += MLP_H * MLP_H;
    std::memcpy(out->b2, p, sizeof(out->b2)); p += MLP_H;
    std::memcpy(out->w3, p, sizeof(out->w3)); p += MLP_H;
    out->b3 = *p;
}

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf(float x)
{
    __hip_bfloat16 b = __float2bfloat16(x);  // round to nearest even
    unsigned short u;
    __builtin_memcpy(&u, &b, 2);
    return (short)u;
}

struct MlpRegs {
    s4 a1[4][2];  // layer-1 weights placed in K-group g, per output block
    f4 c1[2];     // b1 as accumulator input
    s4 a2[2][2];  // layer-2 weight blocks [out block][k block]
    f4 c2[2];     // b2 as accumulator input
    f4 w3[2];
    float b3;
};

__device__ __forceinline__ void load_regs(const MlpDevice *m, int grp, int col, MlpRegs &R)
{
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int j = 0; j < 4; ++j) R.a1[g][mb][j] = grp == g ? bf(m->w1[16 * mb + col][j]) : (short)0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            R.c1[mb][j] = m->b1[16 * mb + 4 * grp + j];
            R.c2[mb][j] = m->b2[16 * mb + 4 * grp + j];
            R.w3[mb][j] = m->w3[16 * mb + 4 * grp + j];
        }
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int j = 0; j < 4; ++j) R.a2[mb][kb][j] = bf(m->w2[16 * mb + col][16 * kb + 4 * grp + j]);
    }
    R.b3 = m->b3;
}

// Network output for the lane's own input x[0..3] (all 64 lanes must be active,
// and every lane's input finite: 0 x inf in a zero block of an operand would
// spread a NaN to the other lanes of the same column).
__device__ __forceinline__ float mlp_wave(const float (&x)[4], const MlpRegs &R, int grp)
{
    const s4 xb = {bf(x[0]), bf(x[1]), bf(x[2]), bf(x[3])};
    float part[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        s4 h1[2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const f4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.a1[g][mb], xb, R.c1[mb], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j) h1[mb][j] = bf(fmaxf(d[j], 0.f));
        }
        float p = 0.f;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            f4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.a2[mb][0], h1[0], R.c2[mb], 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.a2[mb][1], h1[1], d, 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j) p += R.w3[mb][j] * fmaxf(d[j], 0.f);
        }
        p += __shfl_xor(p, 16, 64);
        p += __shfl_xor(p, 32, 64);
        part[g] = p;
    }
    const float y = grp == 0 ? part[0] : (grp == 1 ? part[1] : (grp == 2 ? part[2] : part[3]));
    return y + R.b3;
}

// sigma from the 5-cell stencil w[0..4] (centre w[2])
__device__ __forceinline__ float learned_sigma(const float (&w)[5], const MlpRegs &R, int grp)
{
    float d[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) d[k] = w[k + 1] - w[k];
    const float s = fmaxf(fmaxf(fabsf(d[0]), fabsf(d[1])), fmaxf(fabsf(d[2]), fabsf(d[3]))) +
                    1e-12f * (fabsf(w[2]) + 1e-30f);
    // The floor term alone (a flat stencil of zeros) is below the FP32 normal
    // range, and 1/s would overflow; every input must stay finite because a
    // NaN or infinite input of one lane reaches the other lanes of its column
    // through the zero blocks of the matrix operands.  Inputs are unchanged
    // wherever s is a normal number and exact zeros for a flat stencil.
    const float rs = 1.0f / fmaxf(s, 1.17549435e-38f);
    float x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = d[k] * rs;
    const float sigma = s * mlp_wave(x, R, grp);
    const float dm = d[1], dp = d[2];
    const float sg = dp > 0.f ? 1.f : -1.f;
    const float lim = 2.f * fminf(fabsf(dm), fabsf(dp));
    const float c = sg * fminf(fmaxf(sg * sigma, 0.f), lim);
    return (dm * dp > 0.f) ? c : 0.f;
}

struct Bc {
    int v[3][2];
};

__device__ __forceinline__ int64_t map1(int64_t i, int64_t n, int lo, int hi, bool &flip)
{
    if (i >= 0 && i < n) return i;
    int64_t m;
    if (i < 0) {
        if (lo == BC_PERIODIC) m = i + n;
        else if (lo == BC_OUTFLOW) m = 0;
        else { m = -1 - i; flip = !flip; }
    } else {
        if (hi == BC_PERIODIC) m = i - n;
        else if (hi == BC_OUTFLOW) m = n - 1;
        else { m = 2 * n - 1 - i; flip = !flip; }
    }
    return m < 0 ? 0 : (m >= n ? n - 1 : m);
}

template <int ND>
__global__ void __launch_bounds__(256) k_learned_slopes(const float *__restrict__ u, float *__restrict__ slopes,
                                                        int64_t nx, int64_t ny, int64_t nz, int64_t vs, int64_t svs,
                                                        float gm1, Bc bc, const MlpDevice *__restrict__ mlp)
{
    constexpr int NP = ND + 2;
    const int lane = threadIdx.x & 63, grp = lane >> 4, col = lane & 15;
    MlpRegs R;
    load_regs(mlp, grp, col, R);
    const int64_t ncell = nx * ny * nz;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = c < ncell;
    const int64_t cc = valid ? c : ncell - 1;
    const int64_t ix = cc % nx, iy = (cc / nx) % ny, iz = cc / (nx * ny);
    const int64_t pos[3] = {ix, iy, iz}, nn[3] = {nx, ny, nz};
#pragma unroll
    for (int q = 0; q < ND; ++q) {
        float W[5][NP];
#pragma unroll
        for (int s = 0; s < 5; ++s) {
            bool flip = false;
            int64_t g[3] = {ix, iy, iz};
            g[q] = map1(pos[q] + s - 2, nn[q], bc.v[q][0], bc.v[q][1], flip);
            const int64_t cell = (g[2] * ny + g[1]) * nx + g[0];
            float uu[NP];
#pragma unroll
            for (int v = 0; v < NP; ++v) uu[v] = u[cell + v * vs];
            const float ir = 1.0f / uu[0];
            float ke = 0.f;
            W[s][0] = uu[0];
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                W[s][1 + d] = uu[1 + d] * ir;
                ke += uu[1 + d] * W[s][1 + d];
            }
            W[s][NP - 1] = gm1 * (uu[NP - 1] - 0.5f * ke);
            if (flip) W[s][1 + q] = -W[s][1 + q];
        }
#pragma unroll
        for (int v = 0; v < NP; ++v) {
            const float w5[5] = {W[0][v], W[1][v], W[2][v], W[3][v], W[4][v]};
            const float sg = learned_sigma(w5, R, grp);
            if (valid) slopes[(int64_t)(q * NP + v) * svs + c] = sg;
        }
    }
}

__global__ void __launch_bounds__(256) k_mlp_forward(const MlpDevice *__restrict__ mlp, const float *__restrict__ x,
                                                     float *__restrict__ y, int64_t batch)
{
    const int lane = threadIdx.x & 63, grp = lane >> 4, col = lane & 15;
    MlpRegs R;
    load_regs(mlp, grp, col, R);
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t ii = i < batch ? i : batch - 1;
    const float xi[4] = {x[4 * ii], x[4 * ii + 1], x[4 * ii + 2], x[4 * ii + 3]};
    const float out = mlp_wave(xi, R, grp);
    if (i < batch) y[i] = out;
}

}  // namespace

hipError_t launch_learned_slopes(const float *u, float *slopes, const int64_t n[3], int64_t vstride, int64_t svs,
                                 int ndim, float gm1, const int bc[3][2], const MlpDevice *mlp, hipStream_t s)
{
    Bc b;
    for (int q = 0; q < 3; ++q) {
        b.v[q][0] = bc[q][0];
        b.v[q][1] = bc[q][1];
    }
    const int64_t ncell = n[0] * n[1] * n[2];
    const dim3 grid((unsigned)((ncell + 255) / 256));
    switch (ndim) {
    case 1: hipLaunchKernelGGL(k_learned_slopes<1>, grid, dim3(256), 0, s, u, slopes, n[0], n[1], n[2], vstride, svs, gm1, b, mlp); break;
    case 2: hipLaunchKernelGGL(k_learned_slopes<2>, grid, dim3(256), 0, s, u, slopes, n[0], n[1], n[2], vstride, svs, gm1, b, mlp); break;
    default: hipLaunchKernelGGL(k_learned_slopes<3>, grid, dim3(256), 0, s, u, slopes, n[0], n[1], n[2], vstride, svs, gm1, b, mlp); break;
    }
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDevice *mlp, const float *x, float *y, int64_t batch, hipStream_t s)
{
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, mlp, x, y, batch);
    return hipGetLastError();
}

}  // namespace hy
