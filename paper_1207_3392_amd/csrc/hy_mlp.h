// Learned slope limiter: device weight block and launchers (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hy {

constexpr int MLP_IN = 4;
constexpr int MLP_H = 32;
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;  // 1249

// FP32 master copy of the network, in the ABI order
// W1[32][4], b1[32], W2[32][32], b2[32], w3[32], b3.
struct MlpDevice {
    float w1[MLP_H][MLP_IN];
    float b1[MLP_H];
    float w2[MLP_H][MLP_H];
    float b2[MLP_H];
    float w3[MLP_H];
    float b3;
    float pad[15];
};

void mlp_pack(const float *flat, MlpDevice *out);

// The network as the slope kernel's lanes hold it: for each of the 64 lanes of
// a wave, the 48 registers of its matrix operands (bf16 weights laid out in the
// lane's MFMA positions) and accumulator inputs (FP32 biases), built once per
// weight upload so the slope kernel loads them instead of converting the FP32
// weights in every workgroup.
// Every pre-activation of the network is scaled by 2^-k (k from the weights,
// so that each lies in [-1/2, 1/2] for any input in [-1, 1]); the kernels
// take the output times up = 2^k.  Power-of-two scaling commutes with every
// rounding involved, so the result is the unscaled network's, bit for bit.
struct MlpImage {
    uint4 lane[64][12];
    float up;
    float pad[63];
};

// Builds *img from *mlp on the device (one wave).
hipError_t launch_mlp_image(const MlpDevice *mlp, MlpImage *img, hipStream_t s);

// Slopes of every (dimension q, variable v, interior cell) of the FP32 state u
// (variable stride vstride) from the network, clamped to the TVD region;
// written to slopes[(q * nv + v) * svs + cell].
hipError_t launch_learned_slopes(const float *u, float *slopes, const int64_t n[3], int64_t vstride, int64_t svs,
                                 int ndim, float gm1, const int bc[3][2], const MlpImage *img, hipStream_t s);

// Network alone on a batch of normalised inputs x (batch, 4) -> y (batch).
hipError_t launch_mlp_forward(const MlpDevice *mlp, const float *x, float *y, int64_t batch, hipStream_t s);

}  // namespace hy
