// train.hip -- training the learned slope limiter on gfx950.
//
// Data: a fine run of the plain method is restricted to a grid four times
// coarser (the averaging of the restriction step, 4^d fine cells per coarse
// cell).  Each (coarse cell, primitive variable, dimension) gives one sample:
// the network inputs are the normalised one-sided differences of the 5-cell
// coarse stencil, and the target is the least-squares slope of the four fine
// sub-cell averages along the dimension (positions -3/8, -1/8, 1/8, 3/8 of the
// coarse cell, slope 0.4 (-3 w1 - w2 + w3 + 3 w4)), clamped to the TVD
// region and divided by the same normalisation s.
//
// Step: each workgroup takes tiles of 64 samples and runs the network forward
// and backward with v_mfma_f32_16x16x16_bf16 on operands staged in LDS
// (weights and activations in bfloat16, accumulation in FP32), accumulating
// its share of the gradient of the mean squared error in FP32; a second
// kernel adds the workgroup partials in a fixed order and a third applies
// Adam to the FP32 master weights.
#include "hy_internal.h"
#include "hy_mlp.h"
#include "hy_train.h"

#include <hip/hip_bf16.h>

#include <cmath>
#include <mutex>

namespace hy {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bfu(float x)
{
    __hip_bfloat16 b = __float2bfloat16(x);
    unsigned short u;
    __builtin_memcpy(&u, &b, 2);
    return u;
}

// ------------------------------------------------------------ data ----

// U: conserved fine state (nv vars, stride vs), nf = fine cells per dim;
// out: coarse primitives (nv, nc) and, per dim q, the four sub-cell slab
// averages of each primitive (q, v, 4, nc) for the target slopes.
template <int ND>
__global__ void __launch_bounds__(256) k_coarsen4(const float *__restrict__ U, int64_t vs, int nfx, int nfy, int nfz,
                                                  float gm1, float *__restrict__ Wc, float *__restrict__ sub,
                                                  int64_t nc)
{
    constexpr int NP = ND + 2;
    const int ncx = nfx / 4, ncy = ND >= 2 ? nfy / 4 : 1, ncz = ND == 3 ? nfz / 4 : 1;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= nc) return;
    const int cx = (int)(c % ncx), cy = (int)((c / ncx) % ncy), cz = (int)(c / ((int64_t)ncx * ncy));
    constexpr int KY = ND >= 2 ? 4 : 1, KZ = ND == 3 ? 4 : 1;
    constexpr float inv = 1.0f / (4 * KY * KZ);
    // restriction: averages of the conserved (balanced) variables over the
    // coarse cell and over each quarter slab along every dimension, then the
    // primitives of those averages
    float acc[NP] = {};
    float slab[3][4][NP] = {};
    for (int kz = 0; kz < KZ; ++kz)
        for (int ky = 0; ky < KY; ++ky)
            for (int kx = 0; kx < 4; ++kx) {
                const int64_t f = ((int64_t)(cz * KZ + kz) * nfy + (cy * KY + ky)) * nfx + (cx * 4 + kx);
#pragma unroll
                for (int v = 0; v < NP; ++v) {
                    const float u = U[f + v * vs];
                    acc[v] += u;
                    slab[0][kx][v] += u;
                    if (ND >= 2) slab[1][ky][v] += u;
                    if (ND == 3) slab[2][kz][v] += u;
                }
            }
    auto prim = [&](const float (&u)[NP], float sc, float (&w)[NP]) {
        float uu[NP];
#pragma unroll
        for (int v = 0; v < NP; ++v) uu[v] = u[v] * sc;
        const float ir = 1.0f / uu[0];
        float ke = 0.f;
        w[0] = uu[0];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            w[1 + d] = uu[1 + d] * ir;
            ke += uu[1 + d] * w[1 + d];
        }
        w[NP - 1] = gm1 * (uu[NP - 1] - 0.5f * ke);
    };
    float w[NP];
    prim(acc, inv, w);
#pragma unroll
    for (int v = 0; v < NP; ++v) Wc[v * nc + c] = w[v];
    const float sinv = 4.0f * inv;  // each slab holds a quarter of the fine cells
#pragma unroll
    for (int q = 0; q < ND; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            prim(slab[q][k], sinv, w);
#pragma unroll
            for (int v = 0; v < NP; ++v) sub[((int64_t)(q * NP + v) * 4 + k) * nc + c] = w[v];
        }
}

// samples from the coarse primitives (periodic coarse grid): x (nsamp, 4),
// target t (nsamp); sample index = (q * NP + v) * nc + c
template <int ND>
__global__ void __launch_bounds__(256) k_samples(const float *__restrict__ Wc, const float *__restrict__ sub, int ncx,
                                                 int ncy, int ncz, float *__restrict__ x, float *__restrict__ t)
{
    constexpr int NP = ND + 2;
    const int64_t nc = (int64_t)ncx * ncy * ncz;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nc * NP * ND) return;
    const int64_t c = i % nc;
    const int qv = (int)(i / nc);
    const int q = qv / NP, v = qv % NP;
    const int cx = (int)(c % ncx), cy = (int)((c / ncx) % ncy), cz = (int)(c / ((int64_t)ncx * ncy));
    float w[5];
    for (int s = 0; s < 5; ++s) {
        int p[3] = {cx, cy, cz};
        const int nn[3] = {ncx, ncy, ncz};
        p[q] = ((p[q] + s - 2) % nn[q] + nn[q]) % nn[q];
        w[s] = Wc[v * nc + ((int64_t)p[2] * ncy + p[1]) * ncx + p[0]];
    }
    float d[4];
    for (int k = 0; k < 4; ++k) d[k] = w[k + 1] - w[k];
    // s as in the limiter; the division uses s raised to the smallest normal
    // FP32 number, so a flat stencil of zeros gives x = t = 0, not 0/0
    const float s = fmaxf(fmaxf(fmaxf(fabsf(d[0]), fabsf(d[1])), fmaxf(fabsf(d[2]), fabsf(d[3]))) +
                              1e-12f * (fabsf(w[2]) + 1e-30f),
                          1.17549435e-38f);
    for (int k = 0; k < 4; ++k) x[i * 4 + k] = d[k] / s;
    const float *sb = sub + (int64_t)(q * NP + v) * 4 * nc;
    const float w1 = sb[c], w2 = sb[nc + c], w3 = sb[2 * nc + c], w4 = sb[3 * nc + c];
    float sg = 0.4f * (-3.f * w1 - w2 + w3 + 3.f * w4);
    const float dm = d[1], dp = d[2];
    const float sgn = dp > 0.f ? 1.f : -1.f;
    sg = (dm * dp > 0.f) ? sgn * fminf(fmaxf(sgn * sg, 0.f), 2.f * fminf(fabsf(dm), fabsf(dp))) : 0.f;
    t[i] = sg / s;
}

// ------------------------------------------------------------ step ----

constexpr int TW = 4;          // waves per workgroup
constexpr int TS = 64;         // samples per wave tile
constexpr int H = MLP_H;       // 32
constexpr int KI = 16;         // layer-1 K, padded from 4

// A fragment of a 16 x 16 block: lane (grp, col) holds element
// (i0 + col, j0 + 4 grp + jj), jj = 0..3, of a bf16 matrix at base[i * si + j * sj]
__device__ __forceinline__ s4 frag(const unsigned short *base, int si, int sj, int i0, int j0, int grp, int col)
{
    s4 r;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) r[jj] = (short)base[(i0 + col) * si + (j0 + 4 * grp + jj) * sj];
    return r;
}

// x rounded to the nearest bfloat16 (ties to even), as a float: the third
// layer's operands, which the inference kernel feeds to the matrix cores
__device__ __forceinline__ float bfr(float x) { return __bfloat162float(__float2bfloat16(x)); }

__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }

// Per-wave LDS: X (64 x 16), H1 (64 x 32), dZ (64 x 32), all bf16.
struct WaveLds {
    unsigned short X[TS * KI];
    unsigned short H1[TS * H];
    unsigned short dZ[TS * H];
    float Z1[TS * H];
    float dy[TS];
};

__global__ void __launch_bounds__(64 * TW) k_train_grad(const MlpDevice *__restrict__ m, const float *__restrict__ x,
                                                        const float *__restrict__ t, const int *__restrict__ idx,
                                                        int64_t batch, float inv_batch, float *__restrict__ partial,
                                                        float *__restrict__ loss_partial)
{
    __shared__ unsigned short sW1[H * KI];  // W1 as (j, k), k padded
    __shared__ unsigned short sW2[H * H];   // W2 as (j, k)
    __shared__ WaveLds wl[TW];
    __shared__ float sg[TW][MLP_NPARAM + 3];

    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, grp = lane >> 4, col = lane & 15;
    for (int i = threadIdx.x; i < H * KI; i += 64 * TW) {
        const int j = i / KI, k = i % KI;
        sW1[i] = k < MLP_IN ? bfu(m->w1[j][k]) : 0;
    }
    for (int i = threadIdx.x; i < H * H; i += 64 * TW) sW2[i] = bfu(m->w2[i / H][i % H]);
    for (int i = lane; i < MLP_NPARAM + 3; i += 64) sg[wv][i] = 0.f;
    __syncthreads();

    WaveLds &L = wl[wv];
    float lsum = 0.f;
    // every wave runs the same number of tile iterations (tiles past the end
    // are empty), so workgroup barriers can order the per-wave LDS traffic
    const int64_t ntile = (batch + TS - 1) / TS;
    const int64_t iters = (ntile + (int64_t)gridDim.x * TW - 1) / ((int64_t)gridDim.x * TW);
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t tile = (it * gridDim.x + blockIdx.x) * TW + wv;
        // ---- stage the sample tile ----
        const int64_t si = tile * TS + lane;
        const bool valid = si < batch;
        const int64_t s = valid ? (int64_t)idx[si] : 0;
        float xs[MLP_IN];
#pragma unroll
        for (int k = 0; k < MLP_IN; ++k) xs[k] = valid ? x[s * 4 + k] : 0.f;
        const float ts = valid ? t[s] : 0.f;
#pragma unroll
        for (int k = 0; k < KI; ++k) L.X[lane * KI + k] = k < MLP_IN ? bfu(xs[k]) : 0;
        __syncthreads();

        // ---- layer 1: Z1 (64 x 32) = X (64 x 16) W1^T + b1 ----
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                f4 c;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) c[jj] = m->b1[16 * nb + col];
                // D[m][n] = sum_k X[m][k] W1[n][k]: A = X (m, k), B(k, n) = W1[n][k]
                const s4 a = frag(L.X, KI, 1, 16 * mb, 0, grp, col);
                s4 b;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) b[jj] = (short)sW1[(16 * nb + col) * KI + 4 * grp + jj];
                // fix the accumulator layout: C[m = 4 grp + jj][n = col] = b1[n]
                const f4 d = mfma(a, b, c);
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int mrow = 16 * mb + 4 * grp + jj, ncol = 16 * nb + col;
                    L.Z1[mrow * H + ncol] = d[jj];
                    L.H1[mrow * H + ncol] = bfu(fmaxf(d[jj], 0.f));
                }
            }
        __syncthreads();

        // ---- layer 2 and 3: Z2 = H1 W2^T + b2; y = w3 . relu(Z2) + b3 ----
        float z2[4][2][4];
        float ypart[4][4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) ypart[mb][jj] = 0.f;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                f4 c;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) c[jj] = m->b2[16 * nb + col];
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    const s4 a = frag(L.H1, H, 1, 16 * mb, 16 * kb, grp, col);
                    s4 b;
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) b[jj] = (short)sW2[(16 * nb + col) * H + 16 * kb + 4 * grp + jj];
                    c = mfma(a, b, c);
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    z2[mb][nb][jj] = c[jj];
                    ypart[mb][jj] += bfr(m->w3[16 * nb + col]) * bfr(fmaxf(c[jj], 0.f));
                }
            }
        }
        // y for sample row r = 16 mb + 4 grp + jj: sum over the 16 lanes of the row group
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                float v = ypart[mb][jj];
                v += __shfl_xor(v, 1, 64);
                v += __shfl_xor(v, 2, 64);
                v += __shfl_xor(v, 4, 64);
                v += __shfl_xor(v, 8, 64);
                ypart[mb][jj] = v + m->b3;
            }
        // residual of this lane's own sample (row = lane): held by the lanes of
        // row group (lane / 4) % 4 in block lane / 16
        {
            float yown = 0.f;
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const float v = __shfl(ypart[mb][jj], 16 * ((lane >> 2) & 3), 64);
                    if ((lane >> 4) == mb && (lane & 3) == jj) yown = v;
                }
            const float r = valid ? yown - ts : 0.f;
            lsum += r * r;
            L.dy[lane] = 2.f * r * inv_batch;
        }
        __syncthreads();

        // ---- backward through layer 3: g_w3, g_b3, dZ2 = dy w3 (Z2 > 0) ----
        float gw3[2] = {0.f, 0.f}, gb3 = 0.f, gb2[2] = {0.f, 0.f};
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int mrow = 16 * mb + 4 * grp + jj;
                const float dyr = L.dy[mrow];
                if (col == 0) gb3 += dyr;
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) {
                    const float zz = z2[mb][nb][jj];
                    gw3[nb] += dyr * bfr(fmaxf(zz, 0.f));
                    const float dz = zz > 0.f ? dyr * bfr(m->w3[16 * nb + col]) : 0.f;
                    gb2[nb] += dz;
                    L.dZ[mrow * H + 16 * nb + col] = bfu(dz);
                }
            }
        __syncthreads();
        // per-lane partials summed over the 4 row groups
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            float v = gw3[nb];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            float u = gb2[nb];
            u += __shfl_xor(u, 16, 64);
            u += __shfl_xor(u, 32, 64);
            if (grp == 0) {
                sg[wv][MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + 16 * nb + col] += v;  // w3
                sg[wv][MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + 16 * nb + col] += u;          // b2
            }
        }
        {
            float v = gb3;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) sg[wv][MLP_NPARAM - 1] += v;
        }

        // ---- g_W2 (32 x 32) = dZ2^T (32 x 64) H1 (64 x 32) ----
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) {
                    // A(j, s) = dZ[s][j]; B(s, k) = H1[s][k]
                    const s4 a = frag(L.dZ, 1, H, 16 * mb, 16 * kb, grp, col);
                    const s4 b = frag(L.H1, 1, H, 16 * nb, 16 * kb, grp, col);
                    c = mfma(a, b, c);
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    sg[wv][MLP_H * MLP_IN + MLP_H + (16 * mb + 4 * grp + jj) * H + 16 * nb + col] += c[jj];
            }

        // ---- dH1 (64 x 32) = dZ2 (64 x 32) W2 (32 x 32); dZ1 = dH1 (Z1 > 0) ----
        float dz1[4][2][4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    const s4 a = frag(L.dZ, H, 1, 16 * mb, 16 * kb, grp, col);
                    // B(j, k) = W2[j][k]: element (k = n0 + col, j = k0 + 4 grp + jj)
                    const s4 b = frag(sW2, 1, H, 16 * nb, 16 * kb, grp, col);
                    c = mfma(a, b, c);
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int mrow = 16 * mb + 4 * grp + jj, ncol = 16 * nb + col;
                    dz1[mb][nb][jj] = L.Z1[mrow * H + ncol] > 0.f ? c[jj] : 0.f;
                }
            }
        __syncthreads();
        float gb1[2] = {0.f, 0.f};
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int mrow = 16 * mb + 4 * grp + jj;
                    gb1[nb] += dz1[mb][nb][jj];
                    L.dZ[mrow * H + 16 * nb + col] = bfu(dz1[mb][nb][jj]);
                }
        __syncthreads();
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            float u = gb1[nb];
            u += __shfl_xor(u, 16, 64);
            u += __shfl_xor(u, 32, 64);
            if (grp == 0) sg[wv][MLP_H * MLP_IN + 16 * nb + col] += u;
        }

        // ---- g_W1 (32 x 16) = dZ1^T (32 x 64) X (64 x 16) ----
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const s4 a = frag(L.dZ, 1, H, 16 * mb, 16 * kb, grp, col);
                const s4 b = frag(L.X, 1, KI, 0, 16 * kb, grp, col);
                c = mfma(a, b, c);
            }
            if (col < MLP_IN) {
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) sg[wv][(16 * mb + 4 * grp + jj) * MLP_IN + col] += c[jj];
            }
        }
        __syncthreads();
    }
    __syncthreads();
    // workgroup partial (fixed wave order)
    for (int i = threadIdx.x; i < MLP_NPARAM; i += 64 * TW) {
        float v = 0.f;
#pragma unroll
        for (int w = 0; w < TW; ++w) v += sg[w][i];
        partial[(int64_t)blockIdx.x * MLP_NPARAM + i] = v;
    }
    // loss partial
    {
        float v = lsum;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        __shared__ float sl[TW];
        if (lane == 0) sl[wv] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            float a = 0.f;
            for (int w = 0; w < TW; ++w) a += sl[w];
            loss_partial[blockIdx.x] = a * inv_batch;
        }
    }
}

// Fixed-order sum of the workgroup partials.  Workgroup g takes parameters
// 64 g .. 64 g + 63 (the workgroup after the last one the loss); its wave w
// sums rows w R .. w R + R - 1 in order (R = nblocks / GR_W rounded up), one
// parameter per lane, and the GR_W wave sums are then added in wave order
// through LDS: the same order on every call, and every wave's loads are
// independent of each other (one pass per row instead of one per parameter
// and row).  With ad.m set, the lane that formed a parameter's gradient also
// takes that parameter's Adam step (elementwise, so no other workgroup waits).
constexpr int GR_W = 16;  // waves per workgroup of the gradient sum

__global__ void __launch_bounds__(64 * GR_W) k_grad_reduce(const float *__restrict__ partial, int nblocks,
                                                           const float *__restrict__ loss_partial,
                                                           float *__restrict__ grad, float *__restrict__ loss,
                                                           AdamStep ad)
{
    __shared__ float sp[GR_W][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const bool is_loss = (int)blockIdx.x == (MLP_NPARAM + 63) / 64;
    const int i = (int)blockIdx.x * 64 + lane;
    const int rows = (nblocks + GR_W - 1) / GR_W;
    const int b0 = w * rows, b1 = min(b0 + rows, nblocks);
    float s = 0.f;
    if (is_loss) {
        if (lane == 0)
            for (int b = b0; b < b1; ++b) s += loss_partial[b];
    } else if (i < MLP_NPARAM) {
        for (int b = b0; b < b1; ++b) s += partial[(int64_t)b * MLP_NPARAM + i];
    }
    sp[w][lane] = s;
    __syncthreads();
    if (w == 0) {
        float g = 0.f;
#pragma unroll
        for (int k = 0; k < GR_W; ++k) g += sp[k][lane];
        if (is_loss) {
            if (lane == 0) *loss = g;
        } else if (i < MLP_NPARAM) {
            grad[i] = g;
            if (ad.m) {
                float *p = reinterpret_cast<float *>(ad.m) + i;  // MlpDevice is the flat parameter vector (ABI order)
                const float a = ad.b1 * ad.m1[i] + ad.ob1 * g;
                const float v = ad.b2 * ad.m2[i] + ad.ob2 * g * g;
                ad.m1[i] = a;
                ad.m2[i] = v;
                *p -= ad.lr * (a * ad.c1) / (sqrtf(v * ad.c2) + ad.eps);
            }
        }
    }
}

}  // namespace

hipError_t launch_coarsen4(const float *U, int64_t vs, int ndim, const int nf[3], float gm1, float *Wc, float *sub,
                           hipStream_t s)
{
    int64_t nc = nf[0] / 4;
    if (ndim >= 2) nc *= nf[1] / 4;
    if (ndim == 3) nc *= nf[2] / 4;
    const dim3 grid((unsigned)((nc + 255) / 256));
    if (ndim == 1) hipLaunchKernelGGL(k_coarsen4<1>, grid, dim3(256), 0, s, U, vs, nf[0], 1, 1, gm1, Wc, sub, nc);
    else if (ndim == 2) hipLaunchKernelGGL(k_coarsen4<2>, grid, dim3(256), 0, s, U, vs, nf[0], nf[1], 1, gm1, Wc, sub, nc);
    else hipLaunchKernelGGL(k_coarsen4<3>, grid, dim3(256), 0, s, U, vs, nf[0], nf[1], nf[2], gm1, Wc, sub, nc);
    return hipGetLastError();
}

hipError_t launch_samples(const float *Wc, const float *sub, int ndim, const int nc[3], float *x, float *t,
                          hipStream_t s)
{
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    const int64_t ns = ncell * (ndim + 2) * ndim;
    const dim3 grid((unsigned)((ns + 255) / 256));
    if (ndim == 1) hipLaunchKernelGGL(k_samples<1>, grid, dim3(256), 0, s, Wc, sub, nc[0], 1, 1, x, t);
    else if (ndim == 2) hipLaunchKernelGGL(k_samples<2>, grid, dim3(256), 0, s, Wc, sub, nc[0], nc[1], 1, x, t);
    else hipLaunchKernelGGL(k_samples<3>, grid, dim3(256), 0, s, Wc, sub, nc[0], nc[1], nc[2], x, t);
    return hipGetLastError();
}

hipError_t launch_train_grad(const MlpDevice *m, const float *x, const float *t, const int *idx, int64_t batch,
                             float *partial, float *loss_partial, int nblocks, float *grad, float *loss,
                             const AdamStep &adam, hipStream_t s)
{
    hipLaunchKernelGGL(k_train_grad, dim3(nblocks), dim3(64 * TW), 0, s, m, x, t, idx, batch, 1.0f / (float)batch,
                       partial, loss_partial);
    hipLaunchKernelGGL(k_grad_reduce, dim3((MLP_NPARAM + 63) / 64 + 1), dim3(64 * GR_W), 0, s, partial, nblocks,
                       loss_partial, grad, loss, adam);
    return hipGetLastError();
}

// Staging of hy_lim_make_samples_noalloc: the coarse primitives and sub-cell
// averages live in this library-owned array instead of a caller scratch.
// Host code never passes the symbol itself to a kernel (on the host it names
// a stand-in, not device memory); it uses the per-device address that
// hipGetSymbolAddress returns.
static __device__ __align__(256) float scratch[SAMPLES_STATIC_BYTES / sizeof(float)];

hipError_t samples_static_scratch(int device, float **ptr)
{
    static std::mutex mu;
    static float *addr[MAX_DEVICES] = {};
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        void *a = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != device) {
            const hipError_t er = hipSetDevice(cur);
            if (e == hipSuccess) e = er;
        }
        if (e != hipSuccess) return e;
        addr[device] = (float *)a;
    }
    *ptr = addr[device];
    return hipSuccess;
}

AdamStep adam_step(MlpDevice *m, float *m1, float *m2, float lr, double b1, double b2, float eps, int step)
{
    AdamStep a{};
    a.m = m;
    a.m1 = m1;
    a.m2 = m2;
    a.lr = lr;
    a.b1 = (float)b1;
    a.b2 = (float)b2;
    a.ob1 = (float)(1.0 - b1);
    a.ob2 = (float)(1.0 - b2);
    a.eps = eps;
    a.c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)step)));
    a.c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)step)));
    return a;
}

}  // namespace hy
