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
// All three layers run as bf16 MFMA with FP32 accumulation; biases enter as
// the accumulator input.  One wave evaluates 64 stencils at a time, one per lane,
// in the transposed orientation H^T = W X^T so that each layer's output
// registers are already the next layer's operand layout:
//   lane l = (grp = l / 16, col = l % 16) owns stencil (batch grp, column col);
//   layer 1: for each batch g, A = W1 placed in K-group g (zeros elsewhere),
//            B = the lanes' own bf16 inputs (K-group = grp), C = b1;
//   layer 2: A = W2 (one K = 32 block per output block), B = relu(H1) as
//            bf16, C = b2;
//   layer 3: A = w3 in every row (K = 32), B = relu(H2) as bf16, C = b3, so
//            every row of the result holds the outputs and each lane reads
//            its own stencil's value without a cross-lane reduction.
// The elementwise work between the layers (ReLU and bf16 packing) bounds the
// kernel, so the third layer is put on the matrix cores rather than the
// vector ALU.
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
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 b2 __attribute__((ext_vector_type(2)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ short bf(float x)
{
    __hip_bfloat16 b = __float2bfloat16(x);  // round to nearest even
    unsigned short u;
    __builtin_memcpy(&u, &b, 2);
    return (short)u;
}

// Four floats to a bf16 MFMA operand, two per conversion instruction
// (round to nearest even, element 0 in the low half).
__device__ __forceinline__ s4 bf4(float a, float b, float c, float d)
{
    const u2 w = {__builtin_bit_cast(unsigned, __builtin_convertvector((f2){a, b}, b2)),
                  __builtin_bit_cast(unsigned, __builtin_convertvector((f2){c, d}, b2))};
    return __builtin_bit_cast(s4, w);
}

// Eight floats to a K = 32 bf16 operand (lane elements jj = 0..7).
__device__ __forceinline__ b8 bf8(const s4 lo, const s4 hi)
{
    const u2 l = __builtin_bit_cast(u2, lo), h = __builtin_bit_cast(u2, hi);
    const u4 w = {l[0], l[1], h[0], h[1]};
    return __builtin_bit_cast(b8, w);
}

// The K = 32 operand of the next layer from the two output blocks of a
// 16-stencil batch: every value packed to bf16 with the conversion's output
// clamped to [0, 1], which for pre-activations of magnitude below 1 (the
// scaled network) is the ReLU of the rounded value, bit for bit: negative
// values and -0 give +0.  The inputs are results of matrix instructions, which
// a vector instruction may read only 12 cycles after they issue, and the
// outputs feed matrix instructions, which may read a vector result only 2
// cycles after it is written; the compiler's hazard tracking does not look
// into inline assembly, so the wait states are part of it.
__device__ __forceinline__ b8 relu_pack_clamped(const f4 lo, const f4 hi)
{
    unsigned r0, r1, r2, r3;
    asm("s_nop 11\n\t"
        "v_cvt_pk_bf16_f32 %0, %4, %5 clamp\n\t"
        "v_cvt_pk_bf16_f32 %1, %6, %7 clamp\n\t"
        "v_cvt_pk_bf16_f32 %2, %8, %9 clamp\n\t"
        "v_cvt_pk_bf16_f32 %3, %10, %11 clamp\n\t"
        "s_nop 1"
        : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3)
        : "v"(lo[0]), "v"(lo[1]), "v"(lo[2]), "v"(lo[3]), "v"(hi[0]), "v"(hi[1]), "v"(hi[2]), "v"(hi[3]));
    const u4 w = {r0, r1, r2, r3};
    return __builtin_bit_cast(b8, w);
}

// Layer 2 runs as one K = 32 product per output block (v_mfma_f32_16x16x32_bf16:
// lane (grp, col) holds A[col][8 grp + jj] and B[8 grp + jj][col], jj = 0..7).
// Its K order is permuted so that B is exactly what layer 1 left in the lane:
// K index 8 grp + jj stands for hidden unit hk(grp, jj) = 4 grp + jj (jj < 4)
// or 16 + 4 grp + jj - 4 (jj >= 4), the units of both layer-1 output blocks.
// Layer 3 uses the same K permutation, with w3 replicated over the 16 rows.
struct MlpRegs {
    s4 a1[4][2];  // layer-1 weights placed in K-group g, per output block
    f4 c1[2];     // b1 as accumulator input
    b8 a2[2];     // layer-2 weights [out block], K permuted as above
    f4 c2[2];     // b2 as accumulator input
    b8 a3;        // w3, K permuted as above, the same in every row
    f4 c3;        // b3 as accumulator input
};

__device__ __forceinline__ float bf_value(float x)
{
    const unsigned u = (unsigned)(unsigned short)bf(x) << 16;
    return __uint_as_float(u);
}

// k with 2^k > 2 max(B1, B2), B1 = max_m sum_j |bf16(W1[m][j])| + |b1[m]|
// (inputs lie in [-1, 1]) and B2 = max_m sum_j |bf16(W2[m][j])| B1 + |b2[m]|
// (0 <= h1 <= B1): then every pre-activation times 2^-k lies in [-1/2, 1/2]
// (the factor 2 covers the FP32 accumulation and bf16 rounding).
__device__ __forceinline__ int mlp_upscale(const MlpDevice *m)
{
    float b1 = 0.f, b2 = 0.f;
    for (int r = 0; r < MLP_H; ++r) {
        float a = fabsf(m->b1[r]);
        for (int j = 0; j < MLP_IN; ++j) a += fabsf(bf_value(m->w1[r][j]));
        b1 = fmaxf(b1, a);
    }
    for (int r = 0; r < MLP_H; ++r) {
        float a = 0.f;
        for (int j = 0; j < MLP_H; ++j) a += fabsf(bf_value(m->w2[r][j]));
        b2 = fmaxf(b2, a * b1 + fabsf(m->b2[r]));
    }
    int e = 0;
    (void)frexpf(2.f * fmaxf(b1, b2), &e);  // 2 max(B1, B2) < 2^e
    return e < 0 ? 0 : e;
}

// The lane's operands of the network scaled by 2^-k (k = mlp_upscale): W1
// and every bias times 2^-k (exact: a power of two), W2 and w3 as they are.
__device__ __forceinline__ void load_regs(const MlpDevice *m, int grp, int col, int k, MlpRegs &R)
{
    const float dn = ldexpf(1.f, -k);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int j = 0; j < 4; ++j) R.a1[g][mb][j] = grp == g ? bf(m->w1[16 * mb + col][j] * dn) : (short)0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            R.c1[mb][j] = m->b1[16 * mb + 4 * grp + j] * dn;
            R.c2[mb][j] = m->b2[16 * mb + 4 * grp + j] * dn;
        }
        const float *w2r = m->w2[16 * mb + col];
        R.a2[mb] = bf8(bf4(w2r[4 * grp], w2r[4 * grp + 1], w2r[4 * grp + 2], w2r[4 * grp + 3]),
                       bf4(w2r[16 + 4 * grp], w2r[17 + 4 * grp], w2r[18 + 4 * grp], w2r[19 + 4 * grp]));
    }
    const float *w3 = m->w3;
    R.a3 = bf8(bf4(w3[4 * grp], w3[4 * grp + 1], w3[4 * grp + 2], w3[4 * grp + 3]),
               bf4(w3[16 + 4 * grp], w3[17 + 4 * grp], w3[18 + 4 * grp], w3[19 + 4 * grp]));
#pragma unroll
    for (int j = 0; j < 4; ++j) R.c3[j] = m->b3 * dn;
}

static_assert(sizeof(MlpRegs) == sizeof(uint4) * 12, "lane image layout");

// Network output for the lane's own input x[0..3] (all 64 lanes must be active,
// and every lane's input finite: 0 x inf in a zero block of an operand would
// spread a NaN to the other lanes of the same column).
// The four 16-stencil batches are independent: each layer is issued for all
// of them before the next, so the matrix instructions of one batch overlap
// the ReLU and packing of another instead of the wave waiting on each result.
// Returns the output of the scaled network (the true output times 1 / up).
__device__ __forceinline__ float mlp_wave(const float (&x)[4], const MlpRegs &R, int grp)
{
    const s4 xb = bf4(x[0], x[1], x[2], x[3]);
    f4 d1[4][2];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
            d1[g][mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.a1[g][mb], xb, R.c1[mb], 0, 0, 0);
    b8 hb[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) hb[g] = relu_pack_clamped(d1[g][0], d1[g][1]);
    f4 d2[4][2];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
            d2[g][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(R.a2[mb], hb[g], R.c2[mb], 0, 0, 0);
    b8 h2[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) h2[g] = relu_pack_clamped(d2[g][0], d2[g][1]);
    float part[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) part[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(R.a3, h2[g], R.c3, 0, 0, 0)[0];
    return grp == 0 ? part[0] : (grp == 1 ? part[1] : (grp == 2 ? part[2] : part[3]));
}

// sigma from the 5-cell stencil w[0..4] (centre w[2]); up as in MlpImage
__device__ __forceinline__ float learned_sigma(const float (&w)[5], const MlpRegs &R, int grp, float up)
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
    const float rs = __builtin_amdgcn_rcpf(fmaxf(s, 1.17549435e-38f));  // 1 ulp
    float x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = d[k] * rs;
    const float sigma = s * (mlp_wave(x, R, grp) * up);  // the product with up is exact
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

// Slopes along one dimension Q from a tile of primitives staged in LDS.
// A workgroup owns 64 cells along x times R rows: for Q = 0 the rows are whole
// x lines (y + ny z) and the tile carries a 2-cell halo along x; for Q = 1, 2
// the rows run along y or z at a fixed z or y and the halo is 2 rows each
// side.  Each cell is read and converted to primitives once per dimension;
// then every wave takes whole (variable, row) batches of 64 stencils, so the
// matrix instructions always run with all lanes holding a real stencil.
constexpr int LS_ROWS = 16;

template <int ND, int Q>
struct LsTile {
    static constexpr int NP = ND + 2;
    static constexpr int R = ND == 1 ? 1 : LS_ROWS;  // rows per tile
    static constexpr int NW = ND == 1 ? 1 : 4;       // waves per workgroup (launch bounds match)
    static constexpr int RA = Q == 0 ? R : R + 4;    // LDS rows
    static constexpr int CA = Q == 0 ? 68 : 64;      // LDS columns
};

template <int ND, int Q>
__global__ void __launch_bounds__(ND == 1 ? 64 : 256)
    k_learned_slopes(const float *__restrict__ u, float *__restrict__ slopes, int nx, int ny, int nz, int64_t vs,
                     int64_t svs, float gm1, Bc bc, const MlpImage *__restrict__ img)
{
    using G = LsTile<ND, Q>;
    constexpr int NP = G::NP, R = G::R, NT = 64 * G::NW, RA = G::RA, CA = G::CA;
    __shared__ float sW[NP][RA][CA];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int grp = lane >> 4, col = lane & 15;
    const int x0 = blockIdx.x * 64;
    const int b0 = blockIdx.y * R;  // first row of the tile
    const int cf = blockIdx.z;      // fixed coordinate (z for Q = 1, y for Q = 2)
    const int nq = Q == 0 ? nx : (Q == 1 ? ny : nz);
    const int nrow = Q == 0 ? ny * nz : nq;
    MlpRegs M;
    __builtin_memcpy(&M, &img->lane[lane][0], sizeof(M));
    const float up = img->up;

    for (int i = tid; i < RA * CA; i += NT) {
        const int r = i / CA, c = i % CA;
        bool flip = false;
        int x, y, z;
        if constexpr (Q == 0) {
            x = (int)map1(x0 - 2 + c, nx, bc.v[0][0], bc.v[0][1], flip);
            const int line = min(b0 + r, nrow - 1);
            y = line % ny;
            z = line / ny;
        } else {
            x = min(x0 + c, nx - 1);
            const int qi = (int)map1(b0 - 2 + r, nq, bc.v[Q][0], bc.v[Q][1], flip);
            y = Q == 1 ? qi : cf;
            z = Q == 1 ? cf : qi;
        }
        const int64_t cell = ((int64_t)z * ny + y) * nx + x;
        float uu[NP];
#pragma unroll
        for (int v = 0; v < NP; ++v) uu[v] = u[cell + v * vs];
        const float ir = 1.0f / uu[0];
        float w[NP], ke = 0.f;
        w[0] = uu[0];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            w[1 + d] = uu[1 + d] * ir;
            ke += uu[1 + d] * w[1 + d];
        }
        w[NP - 1] = gm1 * (uu[NP - 1] - 0.5f * ke);
        if (flip) w[1 + Q] = -w[1 + Q];
#pragma unroll
        for (int v = 0; v < NP; ++v) sW[v][r][c] = w[v];
    }
    __syncthreads();

    const int x = x0 + lane;
    for (int k = wv; k < NP * R; k += G::NW) {  // wave-uniform
        const int v = k / R, r = k % R;
        float w5[5];
#pragma unroll
        for (int s5 = 0; s5 < 5; ++s5) w5[s5] = Q == 0 ? sW[v][r][lane + s5] : sW[v][r + s5][lane];
        const float sg = learned_sigma(w5, M, grp, up);
        const int rowi = b0 + r;
        if (x < nx && rowi < nrow) {
            // a variable's slope array is below 4 GiB (checked on the host):
            // 32-bit byte offsets from its (wave-uniform) base
            unsigned cell;
            if constexpr (Q == 0) cell = (unsigned)rowi * (unsigned)nx + (unsigned)x;
            else if constexpr (Q == 1) cell = ((unsigned)cf * (unsigned)ny + (unsigned)rowi) * (unsigned)nx + (unsigned)x;
            else cell = ((unsigned)rowi * (unsigned)ny + (unsigned)cf) * (unsigned)nx + (unsigned)x;
            char *base = (char *)(slopes + (int64_t)(Q * NP + v) * svs);
            *(float *)(base + cell * 4u) = sg;
        }
    }
}

template <int ND, int Q>
void ls_launch(const float *u, float *slopes, int nx, int ny, int nz, int64_t vs, int64_t svs, float gm1, const Bc &b,
               const MlpImage *img, hipStream_t s)
{
    using G = LsTile<ND, Q>;
    const unsigned gx = (unsigned)((nx + 63) / 64);
    const unsigned gy = (unsigned)(Q == 0 ? (ny * nz + G::R - 1) / G::R : ((Q == 1 ? ny : nz) + G::R - 1) / G::R);
    const unsigned gz = (unsigned)(Q == 0 ? 1 : (Q == 1 ? nz : ny));
    hipLaunchKernelGGL((k_learned_slopes<ND, Q>), dim3(gx, gy, gz), dim3(64 * G::NW), 0, s, u, slopes, nx, ny, nz, vs,
                       svs, gm1, b, img);
}

__global__ void __launch_bounds__(64) k_mlp_image(const MlpDevice *__restrict__ mlp, MlpImage *__restrict__ img)
{
    const int lane = threadIdx.x, grp = lane >> 4, col = lane & 15;
    const int k = mlp_upscale(mlp);
    MlpRegs R;
    load_regs(mlp, grp, col, k, R);
    __builtin_memcpy(&img->lane[lane][0], &R, sizeof(R));
    if (lane == 0) img->up = ldexpf(1.f, k);
}

__global__ void __launch_bounds__(256) k_mlp_forward(const MlpDevice *__restrict__ mlp, const float *__restrict__ x,
                                                     float *__restrict__ y, int64_t batch)
{
    const int lane = threadIdx.x & 63, grp = lane >> 4, col = lane & 15;
    const int k = mlp_upscale(mlp);
    const float up = ldexpf(1.f, k);
    MlpRegs R;
    load_regs(mlp, grp, col, k, R);
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t ii = i < batch ? i : batch - 1;
    const float xi[4] = {x[4 * ii], x[4 * ii + 1], x[4 * ii + 2], x[4 * ii + 3]};
    const float out = mlp_wave(xi, R, grp) * up;
    if (i < batch) y[i] = out;
}

}  // namespace

hipError_t launch_learned_slopes(const float *u, float *slopes, const int64_t n[3], int64_t vstride, int64_t svs,
                                 int ndim, float gm1, const int bc[3][2], const MlpImage *img, hipStream_t s)
{
    Bc b;
    for (int q = 0; q < 3; ++q) {
        b.v[q][0] = bc[q][0];
        b.v[q][1] = bc[q][1];
    }
    const int nx = (int)n[0], ny = (int)n[1], nz = (int)n[2];
    switch (ndim) {
    case 1: ls_launch<1, 0>(u, slopes, nx, ny, nz, vstride, svs, gm1, b, img, s); break;
    case 2:
        ls_launch<2, 0>(u, slopes, nx, ny, nz, vstride, svs, gm1, b, img, s);
        ls_launch<2, 1>(u, slopes, nx, ny, nz, vstride, svs, gm1, b, img, s);
        break;
    default:
        ls_launch<3, 0>(u, slopes, nx, ny, nz, vstride, svs, gm1, b, img, s);
        ls_launch<3, 1>(u, slopes, nx, ny, nz, vstride, svs, gm1, b, img, s);
        ls_launch<3, 2>(u, slopes, nx, ny, nz, vstride, svs, gm1, b, img, s);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_mlp_image(const MlpDevice *mlp, MlpImage *img, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_image, dim3(1), dim3(64), 0, s, mlp, img);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDevice *mlp, const float *x, float *y, int64_t batch, hipStream_t s)
{
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, mlp, x, y, batch);
    return hipGetLastError();
}

}  // namespace hy
