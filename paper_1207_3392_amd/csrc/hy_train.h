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
// One Adam step (Kingma & Ba) on the parameter vector m with moments m1, m2:
// b1, b2 the decay rates and ob1 = 1 - b1, ob2 = 1 - b2, each rounded to
// FP32 from its FP64 value; c1, c2 the bias corrections 1 / (1 - b^step),
// formed in FP64 (in FP32, 1 - 0.999^t cancels to a few significant digits
// at small t).  m == nullptr: no step.
struct AdamStep {
    MlpDevice *m;
    float *m1, *m2;
    float lr, b1, b2, ob1, ob2, eps, c1, c2;
};
AdamStep adam_step(MlpDevice *m, float *m1, float *m2, float lr, double b1, double b2, float eps, int step);

// The gradient of the loss over the batch (per-workgroup partials, then their
// fixed-order sum into grad and loss) and, when adam.m is set, the Adam step
// on it, applied by the workgroups that form the sum.
hipError_t launch_train_grad(const MlpDevice *m, const float *x, const float *t, const int *idx, int64_t batch,
                             float *partial, float *loss_partial, int nblocks, float *grad, float *loss,
                             const AdamStep &adam, hipStream_t s);

}  // namespace hy
