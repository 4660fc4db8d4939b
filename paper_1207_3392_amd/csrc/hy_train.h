// Learned-limiter training: launchers (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hy_mlp.h"

namespace hy {

constexpr int TRAIN_BLOCKS = 256;

// The static staging array of the allocation-free sample entry point: bytes
// per GPU, and the devices it serves.
constexpr size_t SAMPLES_STATIC_BYTES = (size_t)64 << 20;
constexpr int MAX_DEVICES = 64;
// Device address of that array on `device` (looked up once per device with
// the device current, then cached).
hipError_t samples_static_scratch(int device, float **ptr);

hipError_t launch_coarsen4(const float *U, int64_t vs, int ndim, const int nf[3], float gm1, float *Wc, float *sub,
                           hipStream_t s);
hipError_t launch_samples(const float *Wc, const float *sub, int ndim, const int nc[3], float *x, float *t,
                          hipStream_t s);
hipError_t launch_train_grad(const MlpDevice *m, const float *x, const float *t, const int *idx, int64_t batch,
                             float *partial, float *loss_partial, int nblocks, float *grad, float *loss, hipStream_t s);
hipError_t launch_adam(MlpDevice *m, const float *grad, float *m1, float *m2, float lr, double b1, double b2,
                       float eps, int step, hipStream_t s);

}  // namespace hy
